"""Collapsed Gauss-Jacobi quadrature on the reference tetrahedron and triangle (oracle).

Test infrastructure only; see ``oracle/__init__``.

The paper uses quadrature-free reference integrals (Sec. 4.1); the oracle
instead integrates at quadrature points, with the Stroud conical-product
rules built from Gauss-Jacobi nodes (scipy's ``roots_jacobi``):

    tetrahedron  x = (1+a)(1-b)(1-c)/8,  y = (1+b)(1-c)/4,  z = (1+c)/2
                 a ~ Gauss-Legendre, b ~ Gauss-Jacobi(1,0), c ~ Gauss-Jacobi(2,0)
                 weight = w_a w_b w_c / 64  (sum = 1/6)
    triangle     s = (1+a)(1-b)/4,  t = (1+b)/2,  weight = w_a w_b / 8  (sum = 1/2)

An n-point-per-direction rule is exact for total degree 2n - 1.

The triangle rule with n = N+1 points per direction also fixes where the
sea-surface displacement eta is stored on a gravity face (one value per
point); its point order is q = j*n + i, i indexing a and j indexing b.
"""
from __future__ import annotations

import numpy as np
from scipy.special import roots_jacobi


def gauss_jacobi(n: int, alpha: float, beta: float):
    x, w = roots_jacobi(n, alpha, beta)
    return np.asarray(x, dtype=np.float64), np.asarray(w, dtype=np.float64)


def tet_rule(n: int):
    """Points [n^3, 3] and weights [n^3] on the reference tetrahedron."""
    a, wa = gauss_jacobi(n, 0.0, 0.0)
    b, wb = gauss_jacobi(n, 1.0, 0.0)
    c, wc = gauss_jacobi(n, 2.0, 0.0)
    A, Bb, C = np.meshgrid(a, b, c, indexing="ij")
    WA, WB, WC = np.meshgrid(wa, wb, wc, indexing="ij")
    x = (1 + A) * (1 - Bb) * (1 - C) / 8.0
    y = (1 + Bb) * (1 - C) / 4.0
    z = (1 + C) / 2.0
    pts = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
    w = (WA * WB * WC).ravel() / 64.0
    return pts, w


def tri_rule(n: int):
    """Points [n^2, 2] (s, t) and weights [n^2] on the reference triangle.

    Point q = j*n + i uses a_i (Gauss-Legendre) and b_j (Gauss-Jacobi(1,0)).
    """
    a, wa = gauss_jacobi(n, 0.0, 0.0)
    b, wb = gauss_jacobi(n, 1.0, 0.0)
    pts = np.empty((n * n, 2))
    w = np.empty(n * n)
    for j in range(n):
        for i in range(n):
            q = j * n + i
            pts[q, 0] = (1 + a[i]) * (1 - b[j]) / 4.0
            pts[q, 1] = (1 + b[j]) / 2.0
            w[q] = wa[i] * wb[j] / 8.0
    return pts, w
