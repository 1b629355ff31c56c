"""Pins of the oracle's Godunov flux and gravity ODE (Sec. 4.2, Sec. 4.3).

Independent checks:
  * same elastic material on both sides: the exact Riemann flux equals the
    textbook flux-vector splitting A+ q- + A- q+ with A+- from numpy's
    eigendecomposition of A-hat(n);
  * the middle state satisfies the characteristic (Rankine-Hugoniot) jump
    relations of the waves on each side;
  * states that already satisfy the elastic-acoustic interface conditions
    are left alone: the flux equals A-hat^- q^- (consistency, Sec. 4.2);
  * the gravity ODE matches its closed form for constant forcing and an
    adaptive high-order integrator (scipy DOP853) for polynomial forcing.
"""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle.physics import normal_jacobian, stress_tensor
from oracle.riemann import godunov_flux, godunov_state, split, gravity_eta_step

ROCK = (3.2404e10, 3.2398e10, 2700.0)          # lam, mu, rho
ROCK2 = (2.0e10, 1.2e10, 2500.0)
WATER = (2.25e9, 0.0, 1000.0)


def _unit(rng):
    n = rng.standard_normal(3)
    return n / np.linalg.norm(n)


def _state(rng):
    q = rng.standard_normal(9)
    q[:6] *= 1e7
    return q


def _mats(m):
    return tuple(np.array(x) for x in m)


def test_same_material_is_flux_vector_splitting():
    rng = np.random.default_rng(0)
    for _ in range(10):
        n = _unit(rng)
        lam, mu, rho = ROCK
        Ah = normal_jacobian(lam, mu, rho, n)
        # A+ and A- by spectral calculus: A-hat is diagonalisable with the five
        # distinct eigenvalues {-cp, -cs, 0, cs, cp}, so f(A-hat) is the Lagrange
        # interpolant of f on them evaluated at A-hat (stress balanced by Zp first).
        cp = math.sqrt((lam + 2 * mu) / rho); cs = math.sqrt(mu / rho)
        ev = np.linalg.eigvals(Ah).real
        np.testing.assert_allclose(np.sort(ev), np.sort([-cp, -cs, -cs, 0, 0, 0, cs, cs, cp]), atol=1e-5)
        D = np.diag([math.sqrt((lam + 2 * mu) * rho)] * 6 + [1.0] * 3)
        Dinv = np.linalg.inv(D)
        As = Dinv @ Ah @ D
        lams = [-cp, -cs, 0.0, cs, cp]

        def fmat(f):
            out = np.zeros((9, 9))
            for i, li in enumerate(lams):
                P = np.eye(9)
                for j, lj in enumerate(lams):
                    if j != i:
                        P = P @ (As - lj * np.eye(9)) / (li - lj)
                out += f(li) * P
            return D @ out @ Dinv

        Ap = fmat(lambda x: max(x, 0.0))
        Am = fmat(lambda x: min(x, 0.0))
        np.testing.assert_allclose(Ap + Am, Ah, atol=1e-9 * np.abs(Ah).max())
        qm, qp = _state(rng), _state(rng)
        F = godunov_flux(qm, qp, n, _mats(ROCK), _mats(ROCK))
        ref = Ap @ qm + Am @ qp
        np.testing.assert_allclose(F, ref, rtol=1e-9, atol=1e-9 * np.abs(ref).max())


@pytest.mark.parametrize("pair", [(ROCK, ROCK2), (ROCK, WATER), (WATER, ROCK), (WATER, WATER)])
def test_middle_state_obeys_jump_relations(pair):
    """Characteristic variables that cross the interface are carried unchanged.

    From the '-' side the right-going invariants s_n - Zp v_n and
    t_t - Zs v_t reach the middle state; from the '+' side the left-going
    s_n + Zp v_n and t_t + Zs v_t. An acoustic side carries no shear
    traction, so the middle state then has t_t = 0.
    """
    rng = np.random.default_rng(1)
    mm, mp = pair
    zpm = math.sqrt((mm[0] + 2 * mm[1]) * mm[2]); zsm = math.sqrt(mm[1] * mm[2])
    zpp = math.sqrt((mp[0] + 2 * mp[1]) * mp[2]); zsp = math.sqrt(mp[1] * mp[2])
    for _ in range(10):
        n = _unit(rng)
        qm, qp = _state(rng), _state(rng)
        if mm[1] == 0:
            qm[3:6] = 0; qm[1] = qm[2] = qm[0]
        if mp[1] == 0:
            qp[3:6] = 0; qp[1] = qp[2] = qp[0]
        vb, tb = godunov_state(qm, qp, n, _mats(mm), _mats(mp))
        snm, ttm, vnm, vtm = split(qm, n)
        snp, ttp, vnp, vtp = split(qp, n)
        snb = tb @ n
        ttb = tb - snb * n
        vnb = vb @ n
        vtb = vb - vnb * n
        scale = 1e7
        assert abs((snb - zpm * vnb) - (snm - zpm * vnm)) < 1e-8 * scale
        assert abs((snb + zpp * vnb) - (snp + zpp * vnp)) < 1e-8 * scale
        if zsm > 0 and zsp > 0:
            np.testing.assert_allclose(ttb - zsm * vtb, ttm - zsm * vtm, atol=1e-8 * scale)
            np.testing.assert_allclose(ttb + zsp * vtb, ttp + zsp * vtp, atol=1e-8 * scale)
        elif zsm > 0:
            np.testing.assert_allclose(ttb, 0.0, atol=1e-8 * scale)
            np.testing.assert_allclose(ttb - zsm * vtb, ttm - zsm * vtm, atol=1e-8 * scale)
        else:
            np.testing.assert_allclose(ttb, 0.0, atol=1e-8 * scale)


def test_interface_consistency():
    """States meeting the interface conditions give F = A-hat^- q^- (Sec. 4.2)."""
    rng = np.random.default_rng(2)
    for mm, mp in [(ROCK, WATER), (WATER, ROCK), (ROCK, ROCK2)]:
        for _ in range(5):
            n = _unit(rng)
            qm = _state(rng)
            snm, ttm, vnm, vtm = split(qm, n)
            if mm[1] == 0 or mp[1] == 0:
                # remove tangential traction on the elastic side: s <- s - (t_t n^T + n t_t^T)
                S = stress_tensor(qm)
                S = S - np.outer(ttm, n) - np.outer(n, ttm)
                qm[[0, 1, 2, 3, 4, 5]] = [S[0, 0], S[1, 1], S[2, 2], S[0, 1], S[1, 2], S[0, 2]]
                snm, ttm, vnm, vtm = split(qm, n)
                assert np.abs(ttm).max() < 1e-6
            if mm[1] == 0:
                qm[1] = qm[2] = qm[0] = snm
                qm[3:6] = 0
            # '+' state with the same traction and velocity
            qp = qm.copy()
            if mp[1] == 0:
                qp[:3] = snm
                qp[3:6] = 0
                if mm[1] > 0:
                    qp[6:9] = vnm * n + rng.standard_normal(3) * 0  # tangential v free
            F = godunov_flux(qm, qp, n, _mats(mm), _mats(mp))
            ref = normal_jacobian(*mm, n) @ qm if False else None
            lam, mu, rho = mm
            ref = normal_jacobian(lam, mu, rho, n) @ qm
            np.testing.assert_allclose(F, ref, rtol=1e-9, atol=1e-9 * np.abs(ref).max())


def test_elastic_acoustic_state_matches_paper_formula():
    """Elastic '-', acoustic '+': middle state in the rotated frame (Sec. 4.2, boundary state)."""
    rng = np.random.default_rng(4)
    lam, mu, rho = ROCK
    zp = math.sqrt((lam + 2 * mu) * rho); zs = math.sqrt(mu * rho)
    zpa = math.sqrt(WATER[0] * WATER[2])
    for _ in range(5):
        n = _unit(rng)
        qm, qp = _state(rng), _state(rng)
        qp[3:6] = 0; qp[1] = qp[2] = qp[0]
        vb, tb = godunov_state(qm, qp, n, _mats(ROCK), _mats(WATER))
        # rotated-frame components with tangents s, t
        s = np.cross(n, [0.3, 0.5, 0.81]); s /= np.linalg.norm(s)
        t = np.cross(n, s)
        Sm = stress_tensor(qm); Sp = stress_tensor(qp)
        w1m, w1p = n @ Sm @ n, n @ Sp @ n
        w4m, w6m = s @ Sm @ n, t @ Sm @ n
        w7m, w7p = qm[6:9] @ n, qp[6:9] @ n
        w8m, w9m = qm[6:9] @ s, qm[6:9] @ t
        a1 = zp * zpa / (zp + zpa) * ((w1m - w1p) / zpa + w7m - w7p)
        np.testing.assert_allclose(tb @ n, w1m - a1, rtol=1e-10)
        np.testing.assert_allclose(vb @ n, w7m - a1 / zp, rtol=1e-10)
        np.testing.assert_allclose([tb @ s, tb @ t], [0.0, 0.0], atol=1e-6)
        np.testing.assert_allclose(vb @ s, w8m - w4m / zs, rtol=1e-10)
        np.testing.assert_allclose(vb @ t, w9m - w6m / zs, rtol=1e-10)


def test_eta_ode_constant_forcing_closed_form():
    a, f, eta0 = 6.5e-3, 0.37, 1.2
    for dt in (1e-3, 0.5, 7.0, 40.0):
        eta, H = gravity_eta_step(np.array([eta0]), np.array([[f]]), a, dt)
        e_ref = f / a + (eta0 - f / a) * math.exp(-a * dt)
        H_ref = f / a * dt + (eta0 - f / a) * (1 - math.exp(-a * dt)) / a
        assert abs(eta[0] - e_ref) < 1e-13 * max(1, abs(e_ref))
        assert abs(H[0] - H_ref) < 1e-12 * max(1, abs(H_ref))


def test_eta_ode_polynomial_forcing_vs_dop853():
    rng = np.random.default_rng(5)
    for N in (2, 5):
        F = rng.standard_normal(N + 1)
        a, eta0, dt = 0.05, 0.3, 2.0

        def f(t):
            return sum(F[m] * t ** m / math.factorial(m) for m in range(N + 1))

        sol = solve_ivp(lambda t, y: [f(t) - a * y[0], y[0]], (0, dt), [eta0, 0.0],
                        method="DOP853", rtol=1e-13, atol=1e-15)
        eta, H = gravity_eta_step(np.array([eta0]), F[None, :], a, dt)
        assert abs(eta[0] - sol.y[0, -1]) < 1e-11
        assert abs(H[0] - sol.y[1, -1]) < 1e-11
