"""Pointwise Godunov flux in the physical frame (oracle).

Test infrastructure only; see ``oracle/__init__``.

The paper solves the Riemann problem at each face exactly (Sec. 4.2): the
jumps across the P and S waves satisfy the Rankine-Hugoniot conditions, and
the middle state w^b is closed by the interface conditions (continuity of
normal traction and normal velocity; zero shear traction at an
elastic-acoustic interface). The numerical flux is A-hat^- q^b.

The oracle writes the same solution in the physical frame with vectors
instead of the rotation T:

    traction t = s n, normal stress s_n = n.t, tangential traction t_t = t - s_n n
    normal velocity v_n = n.v, tangential velocity v_t = v - v_n n
    alpha_1 = Zp- Zp+/(Zp- + Zp+) ((s_n- - s_n+)/Zp+ + v_n- - v_n+)
    s_n^b = s_n- - alpha_1,  v_n^b = v_n- - alpha_1/Zp-        (boundary-state eq.)

Tangential part (the paper prints only the elastic(-)/acoustic(+) case; the
elastic-elastic case is the same characteristic argument with S waves on both
sides, and the acoustic(-) side needs no tangential state since mu- = 0):

    both sides elastic:  alpha_t = Zs- Zs+/(Zs- + Zs+) ((t_t- - t_t+)/Zs+ + v_t- - v_t+)
                         t_t^b = t_t- - alpha_t,  v_t^b = v_t- - alpha_t/Zs-
    elastic(-), fluid(+): t_t^b = 0,  v_t^b = v_t- - t_t-/Zs-
    fluid(-):             t_t^b = 0

The flux is A-hat^-(n) q^b, which depends on q^b only through v^b and the
traction s^b n:
    stress rows   -[lam- (v^b.n) delta_ij + mu- (v^b_i n_j + v^b_j n_i)]
    velocity rows -(s^b n)/rho-
"""
from __future__ import annotations

import numpy as np

from .physics import VOIGT, stress_tensor


def flux_of_state(lam, mu, rho, n, v, t):
    """A-hat(n) q for a state given by velocity v[...,3] and traction t = s n [...,3]."""
    vn = np.einsum("...i,...i->...", v, n)
    F = np.zeros(v.shape[:-1] + (9,))
    for (i, j), s in VOIGT.items():
        if i > j:
            continue
        val = -(mu * (v[..., i] * n[..., j] + v[..., j] * n[..., i]))
        if i == j:
            val = val - lam * vn
        F[..., s] = val
    F[..., 6:9] = -t / rho[..., None]
    return F


def split(q, n):
    """(s_n, t_t, v_n, v_t) of states q[..., 9] on normals n[..., 3]."""
    S = stress_tensor(q)
    t = np.einsum("...ij,...j->...i", S, n)
    sn = np.einsum("...i,...i->...", t, n)
    tt = t - sn[..., None] * n
    v = q[..., 6:9]
    vn = np.einsum("...i,...i->...", v, n)
    vt = v - vn[..., None] * n
    return sn, tt, vn, vt


def godunov_state(qm, qp, n, matm, matp):
    """Middle state (v^b, t^b) seen from the '-' side.

    qm, qp: [..., 9] states; n: [..., 3] unit normal from - to +;
    matm, matp: tuples (lam, mu, rho) of arrays broadcastable to qm[..., 0].
    Returns v^b [..., 3] and traction t^b [..., 3].
    """
    lm, mm, rm = matm
    lp, mp, rp = matp
    zpm = np.sqrt((lm + 2 * mm) * rm)
    zpp = np.sqrt((lp + 2 * mp) * rp)
    zsm = np.sqrt(mm * rm)
    zsp = np.sqrt(mp * rp)
    snm, ttm, vnm, vtm = split(qm, n)
    snp, ttp, vnp, vtp = split(qp, n)

    a1 = zpm * zpp / (zpm + zpp) * ((snm - snp) / zpp + vnm - vnp)
    snb = snm - a1
    vnb = vnm - a1 / zpm

    ela_m = zsm > 0
    ela_p = zsp > 0
    both = ela_m & ela_p
    safe_zsp = np.where(zsp > 0, zsp, 1.0)
    safe_zsm = np.where(zsm > 0, zsm, 1.0)
    at = (zsm * zsp / np.where(both, zsm + zsp, 1.0))[..., None] * (
        (ttm - ttp) / safe_zsp[..., None] + vtm - vtp)
    ttb_both = ttm - at
    vtb_both = vtm - at / safe_zsm[..., None]
    vtb_half = vtm - ttm / safe_zsm[..., None]

    ttb = np.where(both[..., None], ttb_both, 0.0)
    vtb = np.where(both[..., None], vtb_both, np.where(ela_m[..., None], vtb_half, vtm))
    vb = vnb[..., None] * n + vtb
    tb = snb[..., None] * n + ttb
    return vb, tb


def godunov_flux(qm, qp, n, matm, matp):
    """Numerical flux A-hat^- q^b (Sec. 4.2, numerical-flux eq.)."""
    vb, tb = godunov_state(qm, qp, n, matm, matp)
    lm, mm, rm = matm
    return flux_of_state(np.broadcast_to(lm, vb.shape[:-1]), np.broadcast_to(mm, vb.shape[:-1]),
                         np.broadcast_to(rm, vb.shape[:-1]), n, vb, tb)


def ghost_state(kind: int, qm):
    """Ghost q+ for weakly imposed boundaries (Sec. 4.3, 'inverse Riemann problem').

    3 absorbing: q+ = 0; 4 rigid wall: v+ = -v-, same stress;
    5 traction-free surface (g = 0): s+ = -s-, same velocity.
    """
    qp = np.array(qm, copy=True)
    if kind == 3:
        qp[...] = 0.0
    elif kind == 4:
        qp[..., 6:9] *= -1.0
    elif kind == 5:
        qp[..., 0:6] *= -1.0
    else:
        raise ValueError(kind)
    return qp


def gravity_eta_step(eta0, F, a, dt, tol=1e-18, max_terms=200):
    """Exact solution of the per-step ODE of the gravity face (Sec. 4.3, coupled ODE).

    d eta/dt = f(t) - a eta,  dH/dt = eta,  eta(0) = eta0, H(0) = 0,
    with f(t) = sum_m F[m] t^m / m! a polynomial (F[..., m] = d^m f/dt^m at 0)
    and a = rho g / Z. The Taylor coefficients e_m = d^m eta/dt^m (0) satisfy
    e_0 = eta0, e_{m+1} = F_m - a e_m (F_m = 0 beyond the given degree), and
    eta(dt) = sum e_m dt^m/m!, H(dt) = sum e_m dt^(m+1)/(m+1)!; the series is
    summed until its terms fall below ``tol`` of the running sums.

    The paper integrates this ODE with a 7th-order Runge-Kutta method; the
    exact solution is the quantity that method approximates.
    Returns (eta(dt), H(dt)).
    """
    eta0 = np.asarray(eta0, dtype=np.float64)
    F = np.asarray(F, dtype=np.float64)
    nF = F.shape[-1]
    e = eta0.copy()
    coef = 1.0  # dt^m / m!
    eta = np.zeros_like(eta0)
    H = np.zeros_like(eta0)
    for m in range(max_terms):
        term_eta = e * coef
        term_H = e * coef * dt / (m + 1)
        eta = eta + term_eta
        H = H + term_H
        if m >= nF and np.all(np.abs(term_eta) <= tol * np.maximum(np.abs(eta), 1e-300)) \
                and np.all(np.abs(term_H) <= tol * np.maximum(np.abs(H), 1e-300)):
            break
        Fm = F[..., m] if m < nF else 0.0
        e = Fm - a * e
        coef = coef * dt / (m + 1)
    return eta, H
