"""Orthonormal Dubiner basis on the reference tetrahedron (oracle).

Test infrastructure only; see ``oracle/__init__``.

The paper expands the solution in Dubiner's modal basis of P_N with
B_N = C(N+3, 3) functions (Sec. 4.1, semi-discrete form and the expansion
below it). The paper does not print the basis; the reading used here is the
standard collapsed-coordinate construction (Dubiner 1991; Sherwin and
Karniadakis):

    reference tetrahedron  {x, y, z >= 0, x + y + z <= 1}
    collapsed coordinates  a = 2x/(1-y-z) - 1,  b = 2y/(1-z) - 1,  c = 2z - 1
    phi_pqr = P_p^(0,0)(a) ((1-b)/2)^p P_q^(2p+1,0)(b) ((1-c)/2)^(p+q) P_r^(2p+2q+2,0)(c)

normalised so that the integral of phi^2 over the reference tetrahedron is 1,
and ordered by (p+q+r, r, q, p) ascending, so the first B_n functions span P_n.

Values are computed from the definition at points strictly inside the
collapsed chart (all quadrature points are). Gradients use complex-step
differentiation of the same definition, which is exact to rounding for
analytic functions.
"""
from __future__ import annotations

import math

import numpy as np


def n_basis(N: int) -> int:
    """B_N = C(N+3, 3), the dimension of P_N in three variables (Sec. 4.1)."""
    return (N + 1) * (N + 2) * (N + 3) // 6


def n_face_basis(N: int) -> int:
    """Dimension of P_N in two variables."""
    return (N + 1) * (N + 2) // 2


def basis_indices(N: int) -> list[tuple[int, int, int]]:
    """(p, q, r) triples in the order (p+q+r, r, q, p) ascending."""
    idx = [(p, q, r) for p in range(N + 1) for q in range(N + 1) for r in range(N + 1)
           if p + q + r <= N]
    idx.sort(key=lambda t: (t[0] + t[1] + t[2], t[2], t[1], t[0]))
    return idx


def jacobi(n: int, alpha: float, beta: float, x):
    """Jacobi polynomial P_n^(alpha,beta)(x) by its three-term recurrence.

    Works for real or complex arrays (needed for complex-step gradients).
    """
    x = np.asarray(x)
    p0 = np.ones_like(x)
    if n == 0:
        return p0
    p1 = 0.5 * (alpha - beta + (alpha + beta + 2.0) * x)
    for k in range(1, n):
        # recurrence for P_{k+1} from P_k and P_{k-1}
        a1 = 2.0 * (k + 1) * (k + alpha + beta + 1) * (2 * k + alpha + beta)
        a2 = (2 * k + alpha + beta + 1) * (alpha * alpha - beta * beta)
        a3 = (2 * k + alpha + beta) * (2 * k + alpha + beta + 1) * (2 * k + alpha + beta + 2)
        a4 = 2.0 * (k + alpha) * (k + beta) * (2 * k + alpha + beta + 2)
        p0, p1 = p1, ((a2 + a3 * x) * p1 - a4 * p0) / a1
    return p1


def norm2(p: int, q: int, r: int) -> float:
    """Integral of the unnormalised phi_pqr^2 over the reference tetrahedron.

    From the Jacobi orthogonality integrals in collapsed coordinates:
    1 / (2 (2p+1) (p+q+1) (2p+2q+2r+3)).
    """
    return 1.0 / (2.0 * (2 * p + 1) * (p + q + 1) * (2 * p + 2 * q + 2 * r + 3))


def eval_basis(N: int, pts) -> np.ndarray:
    """phi_l at points ``pts`` [n, 3]; returns [n, B] (complex if pts is complex)."""
    pts = np.asarray(pts)
    x, y, z = pts[:, 0], pts[:, 1], pts[:, 2]
    a = 2.0 * x / (1.0 - y - z) - 1.0
    b = 2.0 * y / (1.0 - z) - 1.0
    c = 2.0 * z - 1.0
    cols = []
    for (p, q, r) in basis_indices(N):
        v = (jacobi(p, 0.0, 0.0, a) * ((1.0 - b) / 2.0) ** p
             * jacobi(q, 2.0 * p + 1.0, 0.0, b) * ((1.0 - c) / 2.0) ** (p + q)
             * jacobi(r, 2.0 * p + 2.0 * q + 2.0, 0.0, c))
        cols.append(v / math.sqrt(norm2(p, q, r)))
    return np.stack(cols, axis=1)


def jacobi_h(n: int, alpha: float, beta: float, num, den):
    """den^n P_n^(alpha,beta)(num / den), a polynomial in (num, den).

    The recurrence of ``jacobi`` multiplied through by den^(k+1); finite where
    den = 0, which is where the collapsed coordinates are singular.
    """
    num = np.asarray(num, dtype=np.float64)
    den = np.asarray(den, dtype=np.float64)
    h0 = np.ones_like(num)
    if n == 0:
        return h0
    h1 = 0.5 * (alpha - beta) * den + 0.5 * (alpha + beta + 2.0) * num
    for k in range(1, n):
        a1 = 2.0 * (k + 1) * (k + alpha + beta + 1) * (2 * k + alpha + beta)
        a2 = (2 * k + alpha + beta + 1) * (alpha * alpha - beta * beta)
        a3 = (2 * k + alpha + beta) * (2 * k + alpha + beta + 1) * (2 * k + alpha + beta + 2)
        a4 = 2.0 * (k + alpha) * (k + beta) * (2 * k + alpha + beta + 2)
        h0, h1 = h1, ((a2 * den + a3 * num) * h1 - a4 * den * den * h0) / a1
    return h1


def eval_basis_closed(N: int, pts) -> np.ndarray:
    """phi_l at points of the closed reference tetrahedron [n, 3] -> [n, B].

    The same functions as ``eval_basis``, written without the division of the
    collapsed coordinates: with a = num_a / den_a, num_a = 2x - (1-y-z),
    den_a = 1-y-z and b = num_b / den_b, num_b = 2y - (1-z), den_b = 1-z,
    the factors ((1-b)/2)^p ((1-c)/2)^(p+q) equal den_a^p den_b^q, so
    phi_pqr = [den_a^p P_p(a)] [den_b^q P_q^(2p+1,0)(b)] P_r^(2p+2q+2,0)(c),
    which holds on the faces, edges and vertices as well (receivers there).
    """
    pts = np.asarray(pts, dtype=np.float64)
    x, y, z = pts[:, 0], pts[:, 1], pts[:, 2]
    da, db = 1.0 - y - z, 1.0 - z
    na, nb_ = 2.0 * x - da, 2.0 * y - db
    c = 2.0 * z - 1.0
    cols = []
    for (p, q, r) in basis_indices(N):
        v = (jacobi_h(p, 0.0, 0.0, na, da) * jacobi_h(q, 2.0 * p + 1.0, 0.0, nb_, db)
             * jacobi(r, 2.0 * p + 2.0 * q + 2.0, 0.0, c))
        cols.append(v / math.sqrt(norm2(p, q, r)))
    return np.stack(cols, axis=1)


_H = 1.0e-30


def eval_grad(N: int, pts) -> np.ndarray:
    """Reference gradients d phi_l / d xi_d at real points; returns [n, B, 3]."""
    pts = np.asarray(pts, dtype=np.float64)
    out = []
    for d in range(3):
        pc = pts.astype(np.complex128)
        pc[:, d] += 1j * _H
        out.append(eval_basis(N, pc).imag / _H)
    return np.stack(out, axis=2)
