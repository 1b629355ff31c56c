"""Dynamic-rupture faces: the friction-limited middle state (oracle).

Test infrastructure only; see ``oracle/__init__``.

Fault boundary condition (Sec. 3, eq. bc-dynrup). With n the unit normal
from the '-' to the '+' side, s = n.sigma.n the normal stress,
tau = (I - n n) sigma n the shear traction and V = (I - n n)(v+ - v-) the
slip rate:

    |tau| <= tau_S,   tau_S V - tau |V| = 0,   tau_S = strength(s, psi),   dpsi/dt = g(|V|, psi)

so the fault is locked while the shear traction is below the strength, and
slips parallel to the traction, with the traction at the strength,
otherwise.

Readings (the paper defers the friction law's details to its references):
  * s and tau are totals: the fault carries a background traction (normal
    stress s0 and shear traction tau0) that the elements' state, a
    perturbation, adds to;
  * strength tau_S = C + f max(0, -s) (stress positive in tension, so
    compression closes the fault; C a cohesion);
  * linear slip weakening, the law of the paper's benchmark (Sec. 6.2):
    f = mu_s - (mu_s - mu_d) min(psi / D_c, 1) with psi the slip path,
    dpsi/dt = |V|;
  * the normal stress and the normal velocity are those of the welded
    interface (Godunov middle state, Sec. 4.2); the shear traction follows from
    the S-wave characteristics of each side,
        tau^b = tau- + Zs- (v-^b - v-_t) = tau+ - Zs+ (v+^b - v+_t),
    which for V = 0 gives the locked traction
        tau_lock = eta (tau-/Zs- + tau+/Zs+ + v+_t - v-_t),  eta = Zs- Zs+ / (Zs- + Zs+),
    and in general V = v+^b - v-^b = (tau_lock - tau^b) / eta;
  * over a time step the traces are taken at the N + 1 Gauss-Legendre points
    of the step, in order; at each point the law uses the slip path reached
    so far, and the point's weight times |V| is then added to it.
"""
from __future__ import annotations

import numpy as np

from .riemann import split

# fault parameters per face: s0, tau0 (x, y, z), mu_s, mu_d, D_c, C
N_PARAMS = 8


def friction_coefficient(psi, mu_s, mu_d, dc):
    """Linear slip weakening: mu_s down to mu_d over the slip path D_c."""
    return mu_s - (mu_s - mu_d) * np.minimum(psi / dc, 1.0)


def fault_state(qm, qp, n, matm, matp, params, psi):
    """Middle state of a fault point (see the module notes).

    qm, qp: [..., 9] states of the two sides; n: [..., 3] unit normal from - to
    +; matm, matp: (lam, mu, rho) arrays broadcastable to qm[..., 0];
    params: [..., 8] fault parameters; psi: [...] slip path so far.
    Returns a dict: s (normal stress of the middle state, perturbation),
    vn (normal velocity), tau (shear traction, perturbation), vm, vp
    (tangential velocities of the two sides), V (slip rate), T (total shear
    traction), S (total normal stress).
    """
    lm, mm, rm = matm
    lp, mp, rp = matp
    zpm, zpp = np.sqrt((lm + 2 * mm) * rm), np.sqrt((lp + 2 * mp) * rp)
    zsm, zsp = np.sqrt(mm * rm), np.sqrt(mp * rp)
    snm, ttm, vnm, vtm = split(qm, n)
    snp, ttp, vnp, vtp = split(qp, n)
    # normal part: the welded interface
    s = (zpp * snm + zpm * snp + zpm * zpp * (vnp - vnm)) / (zpm + zpp)
    vn = (zpm * vnm + zpp * vnp + snp - snm) / (zpm + zpp)
    # shear part
    eta = zsm * zsp / (zsm + zsp)
    lock = eta[..., None] * (ttm / zsm[..., None] + ttp / zsp[..., None] + vtp - vtm)
    s0 = params[..., 0]
    tau0 = params[..., 1:4]
    tau0 = tau0 - np.einsum("...i,...i->...", tau0, n)[..., None] * n  # the shear part only
    mu_s, mu_d, dc, coh = (params[..., k] for k in range(4, 8))
    S = s0 + s
    strength = coh + friction_coefficient(psi, mu_s, mu_d, dc) * np.maximum(0.0, -S)
    T = tau0 + lock
    mag = np.sqrt(np.einsum("...i,...i->...", T, T))
    slip = mag > strength
    # below the strength the point is locked: tau = tau_lock and V = 0 exactly
    # (|tau| < tau_S in tau_S V = tau |V| leaves only V = 0)
    ratio = np.where(slip, strength / np.where(slip, mag, 1.0), 1.0)
    Tb = ratio[..., None] * T
    tau = np.where(slip[..., None], Tb - tau0, lock)
    V = np.where(slip[..., None], (lock - tau) / eta[..., None], 0.0)
    vm = vtm + (tau - ttm) / zsm[..., None]
    vp = vtp - (tau - ttp) / zsp[..., None]
    return dict(s=s, vn=vn, tau=tau, vm=vm, vp=vp, V=V, T=Tb, S=S)
