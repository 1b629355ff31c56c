"""Closed-form solutions used to pin the oracle (test infrastructure only).

Plane waves of the velocity-stress system (Sec. 3), the acoustic-gravity
standing wave of a water layer with the linearised sea-surface condition
(Sec. 3, ocean model and gravity boundary condition), and the normal
incidence of a P wave on an elastic-acoustic interface.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.optimize import brentq


def eigenstate(lam, mu, rho, n, v, c):
    """State r = (s, v) with A-hat(n) r = c r for a given velocity polarisation.

    From the velocity rows -s n / rho = c v and the stress rows
    c s = -[lam (v.n) I + mu (v n^T + n v^T)] of A-hat(n) r = c r.
    """
    n = np.asarray(n, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    S = -(lam * np.dot(v, n) * np.eye(3) + mu * (np.outer(v, n) + np.outer(n, v))) / c
    return np.array([S[0, 0], S[1, 1], S[2, 2], S[0, 1], S[1, 2], S[0, 2], v[0], v[1], v[2]])


def plane_wave(lam, mu, rho, m, a_p=1.0, a_s=1.0, pol_angle=0.3):
    """q(x, t) = a_P r_P sin(k (n.x - c_p t)) + a_S r_S sin(k (n.x - c_s t)).

    k = 2 pi |m| and n = m / |m| for an integer vector m (periodic on the unit cube).
    Returns a function (x [n, 3], t) -> q [n, 9].
    """
    m = np.asarray(m, dtype=np.float64)
    k = 2 * math.pi * np.linalg.norm(m)
    n = m / np.linalg.norm(m)
    cp = math.sqrt((lam + 2 * mu) / rho)
    cs = math.sqrt(mu / rho)
    t1 = np.cross(n, [0.12, 0.34, 0.93])
    t1 /= np.linalg.norm(t1)
    t2 = np.cross(n, t1)
    vs = math.cos(pol_angle) * t1 + math.sin(pol_angle) * t2
    rP = eigenstate(lam, mu, rho, n, n, cp)
    rS = eigenstate(lam, mu, rho, n, vs, cs)

    def q(x, t):
        ph = x @ n
        return (a_p * np.sin(k * (ph - cp * t))[:, None] * rP[None, :]
                + a_s * np.sin(k * (ph - cs * t))[:, None] * rS[None, :])

    return q


class StandingWave:
    """Acoustic-gravity standing wave in water of depth H over a rigid bottom.

    p   = P cos(kx) cosh(g_(z+H)) cos(wt)
    v_x = P k / (rho w) sin(kx) cosh(g_(z+H)) sin(wt)
    v_z = -P g_ / (rho w) cos(kx) sinh(g_(z+H)) sin(wt)
    eta = P / (rho g) cos(kx) cosh(g_ H) cos(wt)
    with w^2 = g g_ tanh(g_ H) and g_^2 = k^2 - w^2 / c^2 (found by bracketing).
    The sea surface is z = 0, stress s = -p I.
    """

    def __init__(self, rho, c, g, H, Lx, P=1.0):
        self.rho, self.c, self.g, self.H, self.P = rho, c, g, H, P
        self.k = 2 * math.pi / Lx

        def disp(w):
            gam = math.sqrt(self.k ** 2 - w ** 2 / c ** 2)
            return w ** 2 - g * gam * math.tanh(gam * H)

        self.w = brentq(disp, 1e-9 * self.k * c, self.k * c * (1 - 1e-12), xtol=1e-15, rtol=1e-15)
        self.gam = math.sqrt(self.k ** 2 - self.w ** 2 / c ** 2)

    def q(self, x, t):
        X, Z = x[:, 0], x[:, 2]
        k, w, gm, rho, P = self.k, self.w, self.gam, self.rho, self.P
        p = P * np.cos(k * X) * np.cosh(gm * (Z + self.H)) * math.cos(w * t)
        vx = P * k / (rho * w) * np.sin(k * X) * np.cosh(gm * (Z + self.H)) * math.sin(w * t)
        vz = -P * gm / (rho * w) * np.cos(k * X) * np.sinh(gm * (Z + self.H)) * math.sin(w * t)
        out = np.zeros((x.shape[0], 9))
        out[:, 0:3] = -p[:, None]
        out[:, 6] = vx
        out[:, 8] = vz
        return out

    def eta(self, x, t):
        return (self.P / (self.rho * self.g) * np.cos(self.k * x[:, 0]) * math.cosh(self.gam * self.H)
                * math.cos(self.w * t))


class NormalIncidence:
    """P pulse in an elastic half-space z < 0 meeting water (z > 0) at normal incidence.

    Incident up-going wave r_i f(z - c1 t), reflected r_r f(-z - c1 t) R,
    transmitted r_t f(z (c1/c2) - c1 t) T, with amplitudes from continuity of
    s_zz and v_z at z = 0 (zero shear holds automatically). f is a Gaussian
    pulse centred at z0 < 0 at t = 0.
    """

    def __init__(self, solid, fluid, z0, width):
        (l1, m1, r1), (l2, m2, r2) = solid, fluid
        self.c1 = math.sqrt((l1 + 2 * m1) / r1)
        self.c2 = math.sqrt((l2 + 2 * m2) / r2)
        ez = np.array([0.0, 0.0, 1.0])
        self.ri = eigenstate(l1, m1, r1, ez, ez, self.c1)       # up-going in the solid
        self.rr = eigenstate(l1, m1, r1, ez, ez, -self.c1)      # down-going in the solid
        self.rt = eigenstate(l2, m2, r2, ez, ez, self.c2)       # up-going in the fluid
        # continuity of s_zz (index 2) and v_z (index 8):
        #   ri + R rr = T rt  in those two components
        M = np.array([[self.rr[2], -self.rt[2]], [self.rr[8], -self.rt[8]]])
        rhs = -np.array([self.ri[2], self.ri[8]])
        self.R, self.T = np.linalg.solve(M, rhs)
        self.z0, self.w = z0, width

    def f(self, s):
        return np.exp(-((s - self.z0) / self.w) ** 2)

    def q(self, x, t):
        z = x[:, 2]
        below = z < 0
        out = np.zeros((x.shape[0], 9))
        zb = z[below]
        out[below] = (self.f(zb - self.c1 * t)[:, None] * self.ri
                      + self.R * self.f(-zb - self.c1 * t)[:, None] * self.rr)
        za = z[~below]
        out[~below] = self.T * self.f(za * self.c1 / self.c2 - self.c1 * t)[:, None] * self.rt
        return out
