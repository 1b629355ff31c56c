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
  * rate-and-state friction with fast velocity weakening, the law of the
    Palu run (Sec. 6.3), in its usual regularised form:
        f(V, psi) = a asinh(V / (2 V0) exp(psi / a)),
        dpsi/dt = -(V / L)(psi - psi_ss(V)),
        psi_ss(V) = a ln(2 V0 / V sinh(f_ss(V) / a)),
        f_ss(V) = f_w + (f_LV(V) - f_w) / (1 + (V / V_w)^8)^(1/8),
        f_LV(V) = f0 - (b - a) ln(V / V0);
    the fault always slips: V >= 0 solves |T| - eta V = f(V, psi) max(0, -s)
    (T the total shear traction of the locked state), and over a part of the
    step of length h at that V the state relaxes exactly toward psi_ss(V):
    psi <- psi_ss + (psi - psi_ss) exp(-V h / L);
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

# fault parameters per face (16): s0, tau0 (x, y, z), then the law's:
#   slip weakening (law 0): mu_s, mu_d, D_c, C
#   rate and state (law 1): a, b, L, V0, f0, f_w, V_w, psi0
# and the law at index 15
N_PARAMS = 16
LAW_SLIP_WEAKENING, LAW_RATE_STATE = 0, 1


def friction_coefficient(psi, mu_s, mu_d, dc):
    """Linear slip weakening: mu_s down to mu_d over the slip path D_c."""
    return mu_s - (mu_s - mu_d) * np.minimum(psi / dc, 1.0)


def rs_friction(V, psi, a, V0):
    """Rate-and-state friction coefficient a asinh(V / (2 V0) exp(psi / a))."""
    return a * np.arcsinh(V / (2.0 * V0) * np.exp(psi / a))


def rs_steady_state(V, a, b, V0, f0, fw, Vw):
    """psi_ss(V) of fast velocity weakening."""
    fLV = f0 - (b - a) * np.log(V / V0)
    fss = fw + (fLV - fw) / (1.0 + (V / Vw) ** 8) ** 0.125
    return a * np.log(2.0 * V0 / V * np.sinh(fss / a))


def rs_slip_rate(T, sigma, eta, psi, a, V0, iters=200):
    """Root V in [0, T / eta] of T - eta V - sigma a asinh(V / (2 V0) exp(psi / a)), by bisection.

    The left side falls strictly with V; bisection to the FP64 resolution of
    the bracket (the library solves the same equation by safeguarded Newton).
    """
    lo = np.zeros_like(T)
    hi = T / eta
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        g = T - eta * mid - sigma * rs_friction(mid, psi, a, V0)
        lo = np.where(g > 0, mid, lo)
        hi = np.where(g > 0, hi, mid)
    return 0.5 * (lo + hi)


def fault_state(qm, qp, n, matm, matp, params, psi, h=0.0):
    """Middle state of a fault point (see the module notes).

    qm, qp: [..., 9] states of the two sides; n: [..., 3] unit normal from - to
    +; matm, matp: (lam, mu, rho) arrays broadcastable to qm[..., 0];
    params: [..., 16] fault parameters; psi: [...] slip path (slip
    weakening) or state (rate and state) so far; h: the length of step this
    point stands for (the rate-and-state state relaxes over it).
    Returns a dict: s (normal stress of the middle state, perturbation),
    vn (normal velocity), tau (shear traction, perturbation), vm, vp
    (tangential velocities of the two sides), V (slip rate), T (total shear
    traction), S (total normal stress), psi (the state after the point:
    for slip weakening unchanged, the caller adds |V| h).
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
    S = s0 + s
    T = tau0 + lock
    mag = np.sqrt(np.einsum("...i,...i->...", T, T))
    law = params[..., 15]
    rs = law == LAW_RATE_STATE
    # slip weakening: locked below the strength (tau = tau_lock and V = 0
    # exactly: |tau| < tau_S in tau_S V = tau |V| leaves only V = 0), else at it
    mu_s, mu_d, dc, coh = (params[..., k] for k in range(4, 8))
    strength = coh + friction_coefficient(psi, mu_s, mu_d, np.where(rs, 1.0, dc)) * np.maximum(0.0, -S)
    slip = (mag > strength) & ~rs
    ratio = np.where(slip, strength / np.where(slip, mag, 1.0), 1.0)
    # rate and state: always sliding, |T| - eta V at the rate-dependent strength
    a, b, L, V0, f0, fw, Vw = (params[..., k] for k in range(4, 11))
    a1, V01 = np.where(rs, a, 1.0), np.where(rs, V0, 1.0)
    vrs = rs_slip_rate(np.where(rs, mag, 0.0), np.maximum(0.0, -S), eta, np.where(rs, psi, 0.0), a1, V01)
    ratio = np.where(rs, np.where(mag > 0, (mag - eta * vrs) / np.where(mag > 0, mag, 1.0), 1.0), ratio)
    moving = slip | rs
    Tb = ratio[..., None] * T
    tau = np.where(moving[..., None], Tb - tau0, lock)
    V = np.where(moving[..., None], (lock - tau) / eta[..., None], 0.0)
    speed = np.sqrt(np.einsum("...i,...i->...", V, V))
    # state of rate and state over the point's share h of the step, at that slip rate
    vpos = np.where(rs & (speed > 0), speed, 1.0)
    pss = rs_steady_state(vpos, a1, np.where(rs, b, 1.0), V01, np.where(rs, f0, 1.0), np.where(rs, fw, 1.0),
                          np.where(rs, Vw, 1.0))
    psi_rs = np.where(speed > 0, pss + (psi - pss) * np.exp(-speed * h / np.where(rs, L, 1.0)), psi)
    psi_new = np.where(rs, psi_rs, psi)
    vm = vtm + (tau - ttm) / zsm[..., None]
    vp = vtp - (tau - ttp) / zsp[..., None]
    return dict(s=s, vn=vn, tau=tau, vm=vm, vp=vp, V=V, T=Tb, S=S, psi=psi_new, rs=rs)
