"""Velocity-stress system and its Jacobians (oracle).

Test infrastructure only; see ``oracle/__init__``.

Unknowns q = (s_xx, s_yy, s_zz, s_xy, s_yz, s_xz, v_x, v_y, v_z) (Sec. 3,
elasticity PDE). The PDE

    d s_ij/dt - lam delta_ij dv_k/dx_k - mu (dv_i/dx_j + dv_j/dx_i) = 0
    rho dv_i/dt - d s_ij/dx_j = 0

is written as q_t + A q_x + B q_y + C q_z = 0 (Sec. 4.1, linear PDE form);
the acoustic ocean is the case mu = 0, lam = K, s_ij = -p delta_ij
(Sec. 4.1, first paragraph). Stress is positive in tension, pressure positive
in compression (Sec. 3).
"""
from __future__ import annotations

import numpy as np

# Voigt index of the symmetric stress component (i, j).
VOIGT = {(0, 0): 0, (1, 1): 1, (2, 2): 2, (0, 1): 3, (1, 0): 3, (1, 2): 4, (2, 1): 4,
         (0, 2): 5, (2, 0): 5}


def jacobians(lam: float, mu: float, rho: float) -> np.ndarray:
    """[3, 9, 9] array (A, B, C), read off the PDE term by term."""
    J = np.zeros((3, 9, 9))
    for d in range(3):          # derivative direction x_d
        # stress rows: - lam delta_ij dv_d/dx_d  - mu (dv_i/dx_j + dv_j/dx_i)
        for i in range(3):
            J[d, VOIGT[(i, i)], 6 + d] += -lam
        for i in range(3):
            for j in range(i, 3):
                s = VOIGT[(i, j)]
                if j == d:
                    J[d, s, 6 + i] += -mu
                if i == d:
                    J[d, s, 6 + j] += -mu
        # velocity rows: - (1/rho) d s_ij / dx_j with j = d
        for i in range(3):
            J[d, 6 + i, VOIGT[(i, d)]] += -1.0 / rho
    return J


def normal_jacobian(lam, mu, rho, n) -> np.ndarray:
    """A-hat(n) = n_x A + n_y B + n_z C."""
    J = jacobians(lam, mu, rho)
    return np.tensordot(np.asarray(n, dtype=np.float64), J, axes=(0, 0))


def stress_tensor(q) -> np.ndarray:
    """Symmetric 3x3 stress tensor(s) from Voigt components; q[..., 9] -> [..., 3, 3]."""
    q = np.asarray(q)
    S = np.empty(q.shape[:-1] + (3, 3), dtype=q.dtype)
    for (i, j), s in VOIGT.items():
        S[..., i, j] = q[..., s]
    return S


def wave_speeds(lam, mu, rho):
    cp = np.sqrt((lam + 2.0 * mu) / rho)
    cs = np.sqrt(mu / rho)
    return cp, cs
