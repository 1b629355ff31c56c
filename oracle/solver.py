"""ADER-DG element update with gravity free surface and clustered LTS (oracle).

Test infrastructure only; see ``oracle/__init__``. Plain FP64, vectorised
over elements with numpy; every integral is evaluated at physical quadrature
points (no precomputed reference stiffness or flux matrices, no rotation T).

Method (Sec. 4 of the paper):
  * semi-discrete DG form on each element with an orthonormal modal basis
    (Sec. 4.1, semi-discrete form); the mass matrix is the identity in the
    reference measure;
  * ADER predictor: Taylor expansion in time whose derivatives come from the
    Cauchy-Kowalevski procedure, each time derivative being the L2 projection
    of -(A q_x + B q_y + C q_z) (Sec. 4.1, Taylor expansion);
  * ADER corrector: the Taylor series integrated over the step and inserted
    into the time-integrated weak form (Sec. 4.1);
  * Godunov flux from the exact Riemann solution (Sec. 4.2), boundary
    conditions through ghost states (Sec. 4.3);
  * gravity free surface: per-point ODE for eta and its time integral H, and
    the time-integrated boundary state (Sec. 4.3, coupled ODE system);
  * rate-2 clustered local time stepping (Sec. 4.4).

Readings where the paper is silent (the design notes list them all):
  * cluster c holds dt_K in [2^c dt_min, 2^(c+1) dt_min), capped at
    max_clusters-1, then lowered until face neighbours differ by at most 1;
  * the gravity ODE is integrated exactly (Taylor series of the linear ODE)
    instead of with a 7th-order Runge-Kutta method;
  * p- on a gravity face is -n.s.n.
"""
from __future__ import annotations

import functools
import math

import numpy as np

from . import basis as bas
from . import quadrature as quad
from .mesh import Geometry, adjacency, ref_face_points, FACE_VERTS
from .physics import jacobians, stress_tensor
from .riemann import godunov_flux, ghost_state, gravity_eta_step, flux_of_state
from .fault import LAW_RATE_STATE, LAW_SLIP_WEAKENING, N_PARAMS, fault_state

FACE_INTERIOR, FACE_PERIODIC, FACE_GRAVITY, FACE_ABSORBING, FACE_WALL, FACE_FREE, FACE_VELOCITY, FACE_FAULT = range(8)


def uplift(sources, x, y, t):
    """Seafloor uplift u(x, y, t) = sum_j A_j exp(-r_j^2 / (2 w_j^2)) S(t / T_j).

    S rises from 0 to 1 over the rise time: S(s) = s - sin(2 pi s) / (2 pi) on
    [0, 1] (zero slope at both ends), 0 before and 1 after. The bottom of the
    solid moves with velocity (0, 0, du/dt) (prescribed-velocity faces).
    """
    u = np.zeros(np.broadcast(x, y).shape)
    for a, cx, cy, w, T in sources:
        s = np.clip(t / T, 0.0, 1.0)
        ramp = s - np.sin(2.0 * np.pi * s) / (2.0 * np.pi)
        u = u + a * np.exp(-((x - cx) ** 2 + (y - cy) ** 2) / (2.0 * w * w)) * ramp
    return u

# tensor contractions written as einsum; 'optimize' lets numpy pair them through BLAS
ein = functools.partial(np.einsum, optimize=True)


def taylor_weights(N: int, a: float, b: float) -> np.ndarray:
    """w_k = (b^(k+1) - a^(k+1)) / (k+1)!: integral over [a, b] of t^k / k!."""
    return np.array([(b ** (k + 1) - a ** (k + 1)) / math.factorial(k + 1) for k in range(N + 1)])


def assign_clusters(dt_elem, nb, max_clusters, tied=None):
    """Rate-2 clustering (Sec. 4.4) with the neighbour-difference rule.

    ``tied`` [E, 4] marks faces whose two elements must share a cluster (the
    two sides of a fault face, which the friction law couples pointwise in
    time): across them the rule is c_K <= c_J instead of c_K <= c_J + 1.
    """
    dt_min = float(dt_elem.min())
    c = np.floor(np.log2(dt_elem / dt_min)).astype(np.int64)
    c = np.clip(c, 0, max_clusters - 1)
    step = np.ones(nb.shape, dtype=np.int64) if tied is None else np.where(tied, 0, 1)
    # lower c_K to c_J + 1 wherever a face neighbour J is more than one cluster
    # finer, until nothing changes (the largest assignment obeying the rule)
    while True:
        nbc = np.where(nb >= 0, c[np.maximum(nb, 0)] + step, max_clusters + 1)
        low = np.minimum(c, nbc.min(axis=1))
        if np.array_equal(low, c):
            break
        c = low
    return c, dt_min


class Oracle:
    """Plain FP64 ADER-DG solver on one mesh.

    Arguments mirror the library's set-up call: vertex coordinates [V, 3],
    tetrahedra [E, 4], face kinds [E, 4], period [3], per-element rho, lambda,
    mu, the polynomial degree N (convergence order N+1), the CFL constant C
    in dt = C/(2N+1) h / c_p, gravity g and the number of LTS clusters.
    """

    def __init__(self, xyz, tet, face_kind, period, rho, lam, mu, N, *, cfl=0.35,
                 g=9.81, max_clusters=1, cluster_of=None, dt_min=None):
        self.N = N
        self.B = bas.n_basis(N)
        self.geo = Geometry(xyz, tet)
        self.face_kind = np.asarray(face_kind, dtype=np.int64)
        self.nb, self.nbf, self.shift = adjacency(tet, face_kind, self.geo.xyz, period)
        self.rho = np.asarray(rho, dtype=np.float64)
        self.lam = np.asarray(lam, dtype=np.float64)
        self.mu = np.asarray(mu, dtype=np.float64)
        self.g = float(g)
        E = self.geo.tet.shape[0]
        self.E = E
        self.A = np.stack([jacobians(self.lam[e], self.mu[e], self.rho[e]) for e in range(E)])
        self.cp = np.sqrt((self.lam + 2 * self.mu) / self.rho)
        self.Zp = self.rho * self.cp

        # quadrature rules and basis tables
        self.vpts, self.vw = quad.tet_rule(N + 2)
        self.phi_v = bas.eval_basis(N, self.vpts)           # [q, B]
        self.dphi_v = bas.eval_grad(N, self.vpts)           # [q, B, 3]
        self.fst, self.fw = quad.tri_rule(N + 2)
        self.phi_f = [bas.eval_basis(N, ref_face_points(i, self.fst)) for i in range(4)]
        self.gst, self.gw = quad.tri_rule(N + 1)
        self.phi_g = [bas.eval_basis(N, ref_face_points(i, self.gst)) for i in range(4)]
        # the uplift forcing of prescribed-velocity faces is not polynomial on
        # a face: its face integrals use a rule of N + 10 points per direction
        self.hst, self.hw = quad.tri_rule(N + 10)
        self.phi_h = [bas.eval_basis(N, ref_face_points(i, self.hst)) for i in range(4)]

        # time steps and clusters (Sec. 4.4)
        self.dt_elem = cfl / (2 * N + 1) * self.geo.h / self.cp
        if cluster_of is None:
            self.cluster, self.dt_min = assign_clusters(self.dt_elem, self.nb, max_clusters,
                                                        tied=self.face_kind == FACE_FAULT)
        else:
            self.cluster = np.asarray(cluster_of, dtype=np.int64)
            self.dt_min = float(self.dt_elem.min())
        if dt_min is not None:
            # a patch cut out of a larger mesh steps with that mesh's dt_min
            self.dt_min = float(dt_min)
        self.n_clusters = int(self.cluster.max()) + 1
        self.members = [np.nonzero(self.cluster == c)[0] for c in range(self.n_clusters)]
        self.pos = np.empty(E, dtype=np.int64)
        for c in range(self.n_clusters):
            self.pos[self.members[c]] = np.arange(self.members[c].size)

        # gravity faces, sorted by (element, local face)
        ge, gf = np.nonzero(self.face_kind == FACE_GRAVITY)
        self.grav_elem, self.grav_face = ge, gf
        if ge.size and np.any(self.mu[ge] != 0.0):
            raise ValueError("gravity face on an elastic element")
        self.eta = np.zeros((ge.size, self.gst.shape[0]))

        self._init_faults()

        self.Q = np.zeros((E, self.B, 9))
        self.uplift_sources = []
        self._nb_cache = {}
        self.time = 0.0
        self.updates = 0

    # ------------------------------------------------------------------
    def _init_faults(self):
        """Dynamic-rupture faces (Sec. 3, fault boundary condition).

        A fault face is listed once, from its '-' side: the element with the
        smaller index. Its points are the equispaced lattice of degree N on
        the '-' face (face parameters (j/N, k/N)), where the friction law is
        applied; the flux there is interpolated on the face by the degree-N
        polynomial through those points. The fault starts locked (infinite
        cohesion) until set_fault gives it parameters.
        """
        N = self.N
        fe, ff = np.nonzero(self.face_kind == FACE_FAULT)
        minus = fe < self.nb[fe, ff]
        fe, ff = fe[minus], ff[minus]
        pe, pf = self.nb[fe, ff], self.nbf[fe, ff]
        if fe.size and (np.any(self.mu[fe] <= 0) or np.any(self.mu[pe] <= 0)):
            raise ValueError("a fault face needs elastic elements on both sides")
        if fe.size and np.any(self.cluster[fe] != self.cluster[pe]):
            raise ValueError("the two sides of a fault face are in different clusters")
        self.fault_elem, self.fault_face = fe, ff
        self.fault_pelem, self.fault_pface = pe, pf
        lat = np.array([(j / N, k / N) for j in range(N + 1) for k in range(N + 1 - j)])
        self.fault_lattice = lat
        self.fault_points = self.geo.face_points(fe, ff, lat)            # [F, nf, 3]
        # interpolation of nodal values to the flux points of either side, in
        # the '-' face's parameters (monomials s^a t^b, a + b <= N)
        pw = [(a, b) for a in range(N + 1) for b in range(N + 1 - a)]
        vander = lambda st: np.stack([st[..., 0] ** a * st[..., 1] ** b for a, b in pw], axis=-1)
        Vinv = np.linalg.inv(vander(lat))
        nF = fe.size
        self.fault_Lm = np.broadcast_to(vander(self.fst) @ Vinv, (nF,) + (self.fst.shape[0], lat.shape[0])).copy()
        xp = self.geo.face_points(pe, pf, self.fst)                        # '+' side flux points
        X = self.geo.X
        fv = np.array(FACE_VERTS)[ff]
        P0 = X[fe, fv[:, 0]]
        U = np.stack([X[fe, fv[:, 1]] - P0, X[fe, fv[:, 2]] - P0], axis=2)  # [F, 3, 2]
        stp = np.einsum("fij,fqj->fqi", np.linalg.pinv(U), xp - P0[:, None, :])
        self.fault_Lp = vander(stp) @ Vinv
        self.fault_params = np.zeros((nF, N_PARAMS))
        self.fault_params[:, 6] = 1.0
        self.fault_params[:, 7] = np.inf
        nf = lat.shape[0]
        self.fault_slip = np.zeros((nF, nf, 3))
        self.fault_psi = np.zeros((nF, nf))
        self.fault_rate = np.zeros((nF, nf, 3))
        self.fault_traction = np.zeros((nF, nf, 3))
        self.fault_normal = np.zeros((nF, nf))

    def set_fault(self, params, law=LAW_SLIP_WEAKENING):
        """Fault parameters per face and the fault at rest (no slip, initial state).

        law 0 (slip weakening): params [F, 8] = s0, tau0 (3), mu_s, mu_d, D_c, C;
        law 1 (rate and state): params [F, 12] = s0, tau0 (3), a, b, L, V0, f0, f_w, V_w, psi0.
        """
        p = np.asarray(params, dtype=np.float64)
        k = 8 if law == LAW_SLIP_WEAKENING else 12
        self.fault_params[:] = 0.0
        self.fault_params[:, :k] = np.broadcast_to(p, (self.fault_params.shape[0], k))
        self.fault_params[:, 15] = law
        self.fault_slip[:] = 0.0
        self.fault_rate[:] = 0.0
        self.fault_psi[:] = self.fault_params[:, 11][:, None] if law == LAW_RATE_STATE else 0.0

    def _fault_fluxes(self, c, own, dt):
        """Face-flux updates of the fault faces of cluster c over its step of length dt.

        Returns (element ids, local faces, dQ contributions) for both sides.
        """
        sel = np.nonzero(self.cluster[self.fault_elem] == c)[0]
        if not sel.size:
            return []
        N = self.N
        xg, wg = np.polynomial.legendre.leggauss(N + 1)
        tj = 0.5 * dt * (xg + 1.0)
        wj = 0.5 * dt * wg
        fact = np.array([math.factorial(k) for k in range(N + 1)], dtype=np.float64)
        out = []
        fe, ff, pe, pf = (a[sel] for a in (self.fault_elem, self.fault_face, self.fault_pelem, self.fault_pface))
        x = self.fault_points[sel]                                           # [m, nf, 3]
        n = self.geo.normal[fe, ff][:, None, :] * np.ones((1, x.shape[1], 1))
        # traces of the time derivatives at the lattice points: [m, N+1, nf, 9]
        tr = []
        for e in (fe, pe):
            # the lattice includes the face's vertices: the closed form of the basis is regular there
            phi = bas.eval_basis_closed(N, self.geo.to_ref(e[:, None], x).reshape(-1, 3)).reshape(e.size, -1, self.B)
            tr.append(ein("mqb,mkbp->mkqp", phi, own[self.pos[e]]))
        one = np.ones(x.shape[1])
        matm = tuple(a[fe][:, None] * one for a in (self.lam, self.mu, self.rho))
        matp = tuple(a[pe][:, None] * one for a in (self.lam, self.mu, self.rho))
        prm = self.fault_params[sel][:, None, :] * np.ones((1, x.shape[1], 1))
        psi = self.fault_psi[sel].copy()
        slip = self.fault_slip[sel].copy()
        acc = {k: 0.0 for k in ("s", "vn", "tau", "vm", "vp")}
        for t, w in zip(tj, wj):
            powk = t ** np.arange(N + 1) / fact                              # q(t) = sum_k D_k t^k / k!
            qm = ein("k,mkqp->mqp", powk, tr[0])
            qp = ein("k,mkqp->mqp", powk, tr[1])
            st = fault_state(qm, qp, n, matm, matp, prm, psi, h=w)
            for k in acc:
                acc[k] = acc[k] + w * st[k]
            speed = np.sqrt(np.einsum("...i,...i->...", st["V"], st["V"]))
            psi = np.where(st["rs"], st["psi"], psi + w * speed)
            slip = slip + w * st["V"]
        self.fault_psi[sel] = psi
        self.fault_slip[sel] = slip
        self.fault_rate[sel] = st["V"]
        self.fault_traction[sel] = st["T"]
        self.fault_normal[sel] = st["S"]
        # time-integrated middle states, their fluxes at the lattice points,
        # interpolated to each side's flux points and integrated
        t_int = acc["s"][..., None] * n + acc["tau"]
        v_m = acc["vn"][..., None] * n + acc["vm"]
        v_p = acc["vn"][..., None] * n + acc["vp"]
        Fm = flux_of_state(*matm, n, v_m, t_int)
        Fp = flux_of_state(*matp, -n, v_p, -t_int)
        for e, f, F, L in ((fe, ff, Fm, self.fault_Lm[sel]), (pe, pf, Fp, self.fault_Lp[sel])):
            scale = 2.0 * self.geo.area[e, f] / self.geo.absdet[e]
            Fq = np.matmul(L, F)                                             # [m, q, 9]
            upd = np.zeros((e.size, self.B, 9))
            for i in range(4):
                s2 = np.nonzero(f == i)[0]
                if s2.size:
                    upd[s2] = scale[s2][:, None, None] * np.matmul((self.phi_f[i] * self.fw[:, None]).T, Fq[s2])
            out.append((e, upd))
        return out

    def predict(self, elems):
        """Cauchy-Kowalevski time derivatives D^0..D^N of elements -> [n, N+1, B, 9]."""
        D = [self.Q[elems]]
        n = elems.size
        nq = self.vw.size
        JinvT = np.swapaxes(self.geo.Jinv[elems], 1, 2)[:, None]          # [n, 1, e, d]
        A_rt = np.transpose(self.A[elems], (0, 1, 3, 2)).reshape(n, 27, 9)  # [n, (e p), r]
        dphi = np.transpose(self.dphi_v, (0, 2, 1)).reshape(nq * 3, self.B)  # [(q d), b]
        proj = (self.phi_v * self.vw[:, None]).T                             # [b, q]
        for _ in range(self.N):
            # reference gradient of q_k at the volume points, then the chain rule
            gref = np.matmul(dphi, D[-1]).reshape(n, nq, 3, 9)               # [n, q, d, p]
            gphys = np.matmul(JinvT, gref)                                   # [n, q, e, p]
            # f = -(A q_x + B q_y + C q_z) at the points, then its L2 projection
            f = -np.matmul(gphys.reshape(n, nq, 27), A_rt)                   # [n, q, r]
            D.append(np.matmul(proj, f))
        return np.stack(D, axis=1)

    def eval_at(self, elems, x, coeff):
        """Evaluate polynomials coeff[n, B, 9] of elements at physical points x[n, q, 3]."""
        xi = self.geo.to_ref(elems[:, None], x)
        n, q = x.shape[:2]
        phi = bas.eval_basis(self.N, xi.reshape(-1, 3)).reshape(n, q, self.B)
        return ein("nqb,nbp->nqp", phi, coeff)

    def _neighbour_basis(self, c, i):
        """Neighbour basis values at the flux points of face i of cluster c's elements.

        The physical flux points (shifted across periodic faces) are mapped
        into each neighbour's reference element; cached since the mesh is fixed.
        """
        key = (c, i)
        if key not in self._nb_cache:
            elems = self.members[c]
            kind = self.face_kind[elems, i]
            inter = np.nonzero((kind == FACE_INTERIOR) | (kind == FACE_PERIODIC))[0]
            x = self.geo.face_points(elems[inter], np.full(inter.size, i), self.fst)
            xs = x + self.shift[elems[inter], i][:, None, :]
            J = self.nb[elems[inter], i]
            xi = self.geo.to_ref(J[:, None], xs)
            n, q = xs.shape[:2]
            self._nb_cache[key] = bas.eval_basis(self.N, xi.reshape(-1, 3)).reshape(n, q, self.B)
        return self._nb_cache[key]

    # ------------------------------------------------------------------
    def _integral(self, hist, elems, a, b):
        """Time integral over [a, b] (integer sub-step units) of elements' expansions."""
        out = np.zeros((elems.size, self.B, 9))
        cl = self.cluster[elems]
        for c in np.unique(cl):
            sel = np.nonzero(cl == c)[0]
            rows = self.pos[elems[sel]]
            for (t0, length, D) in hist[c]:
                lo, hi = max(a, t0), min(b, t0 + length)
                if hi <= lo:
                    continue
                w = taylor_weights(self.N, (lo - t0) * self.dt_min, (hi - t0) * self.dt_min)
                out[sel] += np.tensordot(w, D[rows], axes=(0, 1))
        return out

    def correct(self, c, hist, t0):
        """Corrector of cluster c over [t0, t0 + 2^c] (sub-step units)."""
        elems = self.members[c]
        length = 1 << c
        dt = length * self.dt_min
        own = hist[c][-1][2][np.arange(elems.size)]
        I = np.tensordot(taylor_weights(self.N, 0.0, dt), own, axes=(0, 1))
        n = elems.size
        nq = self.vw.size
        # volume term: sum_q w_q grad_x(phi_l) . (A_e I)(x_q)
        Iq = np.matmul(self.phi_v, I)                                        # [n, q, p]
        A_p = np.transpose(self.A[elems], (0, 3, 1, 2)).reshape(n, 9, 27)   # [n, p, (e r)]
        AI = np.matmul(Iq, A_p).reshape(n, nq, 3, 9)                         # [n, q, e, r]
        G = np.matmul(self.geo.Jinv[elems][:, None], AI)                     # [n, q, d, r]
        Wd = (np.transpose(self.dphi_v, (0, 2, 1)) * self.vw[:, None, None]).reshape(nq * 3, self.B).T
        dQ = np.matmul(Wd, G.reshape(n, nq * 3, 9))                          # [n, b, r]

        matm = (self.lam[elems], self.mu[elems], self.rho[elems])
        for i in range(4):
            kind = self.face_kind[elems, i]
            scale = 2.0 * self.geo.area[elems, i] / self.geo.absdet[elems]
            n = self.geo.normal[elems, i]
            # ordinary faces at the (N+2)^2 flux points
            Im = np.matmul(self.phi_f[i], I)
            Ip = np.zeros_like(Im)
            lp, mp, rp = (a.copy() for a in matm)
            inter = np.nonzero((kind == FACE_INTERIOR) | (kind == FACE_PERIODIC))[0]
            if inter.size:
                J = self.nb[elems[inter], i]
                Inb = self._integral(hist, J, t0, t0 + length)
                Ip[inter] = np.matmul(self._neighbour_basis(c, i), Inb)
                lp[inter], mp[inter], rp[inter] = self.lam[J], self.mu[J], self.rho[J]
            for k in (FACE_ABSORBING, FACE_WALL, FACE_FREE):
                sel = np.nonzero(kind == k)[0]
                if sel.size:
                    Ip[sel] = ghost_state(k, Im[sel])
            vel = np.nonzero(kind == FACE_VELOCITY)[0]
            if vel.size:
                # prescribed velocity v_b = (0, 0, du/dt): ghost v+ = 2 v_b - v-, same stress
                # (Sec. 4.3 ghost states); the flux is linear in the ghost, so the wall part is
                # taken here and the 2 v_b part below
                Ip[vel] = ghost_state(FACE_WALL, Im[vel])
            nq = Im.shape[1]
            nn = np.broadcast_to(n[:, None, :], (n.shape[0], nq, 3))
            F = godunov_flux(Im, Ip, nn,
                             tuple(m[:, None] * np.ones(nq) for m in matm),
                             (lp[:, None] * np.ones(nq), mp[:, None] * np.ones(nq),
                              rp[:, None] * np.ones(nq)))
            F[(kind == FACE_GRAVITY) | (kind == FACE_FAULT)] = 0.0
            dQ -= scale[:, None, None] * np.matmul((self.phi_f[i] * self.fw[:, None]).T, F)
            if vel.size:
                # 2 v_b integrated over the step, 2 (u(t1) - u(t0)), as the neighbour trace
                # (zero own trace); the face integral with the high-order rule
                x = self.geo.face_points(elems[vel], np.full(vel.size, i), self.hst)
                ta = self.time + t0 * self.dt_min
                du = (uplift(self.uplift_sources, x[..., 0], x[..., 1], ta + dt)
                      - uplift(self.uplift_sources, x[..., 0], x[..., 1], ta))
                nh = self.hw.size
                Pp = np.zeros((vel.size, nh, 9))
                Pp[..., 8] = 2.0 * du
                omat = tuple(m[vel][:, None] * np.ones(nh) for m in matm)
                nv = np.broadcast_to(n[vel][:, None, :], (vel.size, nh, 3))
                Fh = godunov_flux(np.zeros_like(Pp), Pp, nv, omat, omat)
                dQ[vel] -= scale[vel][:, None, None] * np.matmul((self.phi_h[i] * self.hw[:, None]).T, Fh)

        # fault faces of this cluster (Sec. 3, friction boundary condition)
        for e, upd in self._fault_fluxes(c, own, dt):
            np.subtract.at(dQ, np.searchsorted(elems, e), upd)

        # gravity faces of this cluster (Sec. 4.3)
        gsel = np.nonzero(self.cluster[self.grav_elem] == c)[0]
        if gsel.size:
            ge = self.grav_elem[gsel]
            gf = self.grav_face[gsel]
            rows = self.pos[ge]
            D = own[rows]                                   # [m, N+1, B, 9]
            for i in range(4):
                s2 = np.nonzero(gf == i)[0]
                if not s2.size:
                    continue
                e = ge[s2]
                Dq = ein("qb,nkbp->nkqp", self.phi_g[i], D[s2])  # [m, N+1, q, 9]
                n = self.geo.normal[e, i]                    # [m, 3]
                S = stress_tensor(Dq)
                pm = -ein("ni,nkqij,nj->nkq", n, S, n)
                vn = ein("ni,nkqi->nkq", n, Dq[..., 6:9])
                Z = self.Zp[e][:, None, None]
                Fm = np.moveaxis(vn + pm / Z, 1, 2)          # [m, q, N+1]
                a = (self.rho[e] * self.g / self.Zp[e])[:, None]
                eta0 = self.eta[gsel[s2]]
                eta1, H = gravity_eta_step(eta0, Fm, a, dt)
                # time-integrated boundary state: int v_n^b = eta1 - eta0, int p^b = rho g H
                nq = eta0.shape[1]
                nn = np.broadcast_to(n[:, None, :], (n.shape[0], nq, 3))
                vb = (eta1 - eta0)[..., None] * nn
                tb = -(self.rho[e][:, None] * self.g * H)[..., None] * nn
                ones = np.ones(nq)
                F = flux_of_state(self.lam[e][:, None] * ones, self.mu[e][:, None] * ones,
                                  self.rho[e][:, None] * ones, nn, vb, tb)
                scale = 2.0 * self.geo.area[e, i] / self.geo.absdet[e]
                upd = scale[:, None, None] * ein("q,qb,nqp->nbp", self.gw, self.phi_g[i], F)
                # elems is sorted; map each gravity face to its row in dQ
                idx = np.searchsorted(elems, e)
                np.subtract.at(dQ, idx, upd)
                self.eta[gsel[s2]] = eta1
        self.Q[elems] += dQ
        self.updates += elems.size

    # ------------------------------------------------------------------
    def macro_step(self):
        """One LTS macro step: 2^(C-1) sub-steps of dt_min (Sec. 4.4)."""
        C = self.n_clusters
        nsub = 1 << (C - 1)
        hist = {c: [] for c in range(C)}
        start = {c: 0 for c in range(C)}
        for s in range(nsub):
            for c in range(C):
                if s % (1 << c) == 0 and self.members[c].size:
                    hist[c].append((s, 1 << c, self.predict(self.members[c])))
                    start[c] = s
            for c in range(C):
                if (s + 1) % (1 << c) == 0 and self.members[c].size:
                    self.correct(c, hist, start[c])
        self.time += nsub * self.dt_min

    def run(self, n_macro: int):
        for _ in range(n_macro):
            self.macro_step()

    # ------------------------------------------------------------------
    def project(self, fn):
        """L2 projection of q0(x) (fn: [n, 3] -> [n, 9]) onto the basis."""
        x = self.geo.x0[:, None, :] + ein("edc,qc->eqd", self.geo.J, self.vpts)
        vals = fn(x.reshape(-1, 3)).reshape(self.E, -1, 9)
        return ein("q,qb,eqp->ebp", self.vw, self.phi_v, vals)

    def eta_points(self):
        """Physical points [F_g, q, 3] where eta is stored."""
        return self.geo.face_points(self.grav_elem, self.grav_face, self.gst)

    def energy(self, Q=None, eta=None):
        """E = sum_K int_K (rho|v|^2/2 + W(s)) + sum_gravity faces int rho g eta^2 / 2."""
        Q = self.Q if Q is None else Q
        eta = self.eta if eta is None else eta
        qv = ein("qb,ebp->eqp", self.phi_v, Q)
        v2 = np.sum(qv[..., 6:9] ** 2, axis=-1)
        S = stress_tensor(qv)
        ss = ein("eqij,eqij->eq", S, S)
        tr = ein("eqii->eq", S)
        lam, mu = self.lam[:, None], self.mu[:, None]
        ela = (mu > 0)
        W_el = (ss - lam / (3 * lam + 2 * mu) * tr ** 2) / (4 * np.where(ela, mu, 1.0))
        p = -tr / 3.0
        W_ac = p ** 2 / (2 * lam)
        W = np.where(ela, W_el, W_ac)
        dens = 0.5 * self.rho[:, None] * v2 + W
        E = float(np.sum(self.geo.absdet[:, None] * self.vw[None, :] * dens))
        if self.grav_elem.size:
            a2 = 2.0 * self.geo.area[self.grav_elem, self.grav_face]
            E += float(np.sum(a2[:, None] * self.gw[None, :] * 0.5 * self.rho[self.grav_elem][:, None]
                              * self.g * eta ** 2))
        return E

    def field_sq_norms(self, Q=None):
        """int over the mesh of q_p^2 for each quantity p (volume quadrature) -> [9]."""
        Q = self.Q if Q is None else Q
        qv = ein("qb,ebp->eqp", self.phi_v, Q)
        return ein("e,q,eqp->p", self.geo.absdet, self.vw, qv ** 2)

    # ------------------------------------------------------------------
    # output at points: receivers, the sea surface and the seafloor (Sec. 6.2)
    def locate(self, points, tol=1e-9):
        """Element and reference coordinates of physical points [n, 3].

        A point belongs to the elements whose barycentric coordinates are all
        >= -tol; of several (a point on a shared face, edge or vertex) the one
        with the lowest element id is taken. Raises if a point is outside.
        """
        points = np.atleast_2d(np.asarray(points, dtype=np.float64))
        elem = np.empty(points.shape[0], dtype=np.int64)
        xi = np.empty((points.shape[0], 3))
        for k, x in enumerate(points):
            ref = np.einsum("edc,ec->ed", self.geo.Jinv, x[None, :] - self.geo.x0)
            bary = np.concatenate([1.0 - ref.sum(axis=1, keepdims=True), ref], axis=1)
            inside = np.nonzero(np.all(bary >= -tol, axis=1))[0]
            if inside.size == 0:
                raise ValueError(f"point {x} is outside the mesh")
            elem[k] = inside[0]
            xi[k] = ref[inside[0]]
        return elem, xi

    def sample(self, points, Q=None):
        """The nine quantities at physical points [n, 3] -> [n, 9] (see locate)."""
        Q = self.Q if Q is None else Q
        elem, xi = self.locate(points)
        phi = bas.eval_basis_closed(self.N, xi)
        return ein("nb,nbp->np", phi, Q[elem])

    def seafloor_faces(self):
        """Elastic-acoustic interface faces seen from the elastic side, sorted by (element, face)."""
        el, fa = [], []
        for e in range(self.E):
            if self.mu[e] == 0.0:
                continue
            for f in range(4):
                j = self.nb[e, f]
                if j >= 0 and self.mu[j] == 0.0:
                    el.append(e)
                    fa.append(f)
        return np.array(el, dtype=np.int64), np.array(fa, dtype=np.int64)

    def face_sample(self, elems, faces, Q=None):
        """The nine quantities of elements elems at the eta-rule points of their faces -> [n, q, 9]."""
        Q = self.Q if Q is None else Q
        out = np.empty((len(elems), self.gst.shape[0], 9))
        for k, (e, f) in enumerate(zip(elems, faces)):
            out[k] = self.phi_g[f] @ Q[e]
        return out

    def evaluate(self, x_elem, xi):
        """Solution at reference points xi[n, 3] of elements x_elem[n] -> [n, 9]."""
        phi = bas.eval_basis(self.N, xi)
        return ein("nb,nbp->np", phi, self.Q[x_elem])
