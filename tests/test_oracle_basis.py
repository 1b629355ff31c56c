"""Pins of the oracle's basis, quadrature and Jacobians against closed forms.

The basis dimension B_N = C(N+3, 3) and the DOF count of the paper's largest
mesh (518 M elements x 56 x 9 = 261 G, Sec. 6) are bookkeeping pins.
"""
import math

import numpy as np
import pytest
from scipy.special import eval_jacobi

from oracle import basis, quadrature
from oracle.mesh import REF_VERTS, FACE_VERTS, ref_face_points
from oracle.physics import jacobians, normal_jacobian

pytestmark = pytest.mark.filterwarnings("ignore")


def test_basis_dimension_and_dof_count():
    assert [basis.n_basis(N) for N in range(7)] == [1, 4, 10, 20, 35, 56, 84]
    for N in range(7):
        assert basis.n_basis(N) == math.comb(N + 3, 3)
        assert len(basis.basis_indices(N)) == basis.n_basis(N)
    # Sec. 6: 518 million elements at degree 5 carry about 261 billion DOF
    assert abs(518e6 * basis.n_basis(5) * 9 / 261e9 - 1.0) < 0.01


def test_jacobi_matches_scipy():
    x = np.linspace(-0.95, 0.95, 11)
    for n in range(8):
        for a in (0, 1, 2, 5, 9, 14):
            np.testing.assert_allclose(basis.jacobi(n, a, 0, x), eval_jacobi(n, a, 0, x),
                                       rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8])
def test_tet_rule_integrates_monomials(n):
    pts, w = quadrature.tet_rule(n)
    for a in range(2 * n):
        for b in range(2 * n - a):
            for c in range(2 * n - a - b):
                exact = math.factorial(a) * math.factorial(b) * math.factorial(c) / math.factorial(a + b + c + 3)
                got = np.sum(w * pts[:, 0] ** a * pts[:, 1] ** b * pts[:, 2] ** c)
                assert abs(got - exact) < 1e-14, (a, b, c)


@pytest.mark.parametrize("n", [1, 2, 4, 7])
def test_tri_rule_integrates_monomials(n):
    pts, w = quadrature.tri_rule(n)
    for a in range(2 * n):
        for b in range(2 * n - a):
            exact = math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)
            got = np.sum(w * pts[:, 0] ** a * pts[:, 1] ** b)
            assert abs(got - exact) < 1e-15, (a, b)


@pytest.mark.parametrize("N", range(0, 7))
def test_orthonormal(N):
    pts, w = quadrature.tet_rule(N + 2)
    phi = basis.eval_basis(N, pts)
    M = phi.T @ (w[:, None] * phi)
    np.testing.assert_allclose(M, np.eye(basis.n_basis(N)), atol=1e-13)


@pytest.mark.parametrize("N", range(0, 7))
def test_hierarchical_degrees(N):
    """The first B_n functions span P_n: phi_l for l < B_n has degree <= n.

    Checked by exactness: a degree-d function restricted to a line is a
    polynomial of degree d in the line parameter, so its (d+1)-th finite
    difference on an equispaced set vanishes.
    """
    rng = np.random.default_rng(1)
    idx = basis.basis_indices(N)
    for _ in range(3):
        p0 = np.array([0.2, 0.15, 0.1]) + 0.05 * rng.random(3)
        d = rng.standard_normal(3)
        d = 0.05 * d / np.linalg.norm(d)
        s = np.arange(N + 3)
        pts = p0[None, :] + s[:, None] * d[None, :]
        phi = basis.eval_basis(N, pts)
        for l, (p, q, r) in enumerate(idx):
            deg = p + q + r
            diff = np.diff(phi[:, l], n=deg + 1)
            assert np.abs(diff).max() < 1e-8 * max(1.0, np.abs(phi[:, l]).max())


@pytest.mark.parametrize("N", [1, 3, 5])
def test_gradient_matches_finite_differences(N):
    pts, _ = quadrature.tet_rule(N + 1)
    g = basis.eval_grad(N, pts)
    h = 1e-6
    for d in range(3):
        pp, pm = pts.copy(), pts.copy()
        pp[:, d] += h
        pm[:, d] -= h
        fd = (basis.eval_basis(N, pp) - basis.eval_basis(N, pm)) / (2 * h)
        np.testing.assert_allclose(g[:, :, d], fd, atol=2e-6 * np.abs(g).max())


@pytest.mark.parametrize("N", [1, 2, 4, 6])
def test_integration_by_parts_on_reference(N):
    """K^d + (K^d)^T equals the boundary integral of phi_k phi_l n_d.

    K^d_kl = int d(phi_k)/d(xi_d) phi_l over the reference tetrahedron; the
    boundary term uses the reference faces (area and outward normal computed
    from the vertices) and the triangle rule through the face parametrisation.
    """
    pts, w = quadrature.tet_rule(N + 2)
    phi = basis.eval_basis(N, pts)
    g = basis.eval_grad(N, pts)
    st, wf = quadrature.tri_rule(N + 2)
    for d in range(3):
        K = np.einsum("q,qk,ql->kl", w, g[:, :, d], phi)
        bnd = np.zeros_like(K)
        for i, (a, b, c) in enumerate(FACE_VERTS):
            cr = np.cross(REF_VERTS[b] - REF_VERTS[a], REF_VERTS[c] - REF_VERTS[a])
            area = 0.5 * np.linalg.norm(cr)
            n = cr / np.linalg.norm(cr)
            if np.dot(n, REF_VERTS[i] - REF_VERTS[a]) > 0:
                n = -n
            pf = basis.eval_basis(N, ref_face_points(i, st))
            bnd += 2 * area * n[d] * np.einsum("q,qk,ql->kl", wf, pf, pf)
        np.testing.assert_allclose(K + K.T, bnd, atol=1e-12)


def _rot(rng):
    Qm, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    return Qm


def test_jacobian_eigenvalues():
    rng = np.random.default_rng(3)
    rho, cp, cs = 2700.0, 6000.0, 3464.0
    mu = rho * cs ** 2
    lam = rho * cp ** 2 - 2 * mu
    for _ in range(5):
        n = rng.standard_normal(3)
        n /= np.linalg.norm(n)
        ev = np.sort(np.linalg.eigvals(normal_jacobian(lam, mu, rho, n)).real)
        np.testing.assert_allclose(ev, np.sort([-cp, -cs, -cs, 0, 0, 0, cs, cs, cp]), atol=1e-6)


def test_jacobians_satisfy_hand_derived_plane_waves():
    """P and S plane waves along each axis, derived from the PDE by hand.

    Along axis a with velocity polarisation b, the wave v_b = f(x_a - c t)
    needs s_ab = -rho c f (and, for P, s_kk = -(lam/c) f for k != a); then
    A-hat(e_a) r = c r for the state vector r.
    """
    rho, lam, mu = 2000.0, 3.0e9, 1.5e9
    cp = np.sqrt((lam + 2 * mu) / rho)
    cs = np.sqrt(mu / rho)
    voigt = {(0, 0): 0, (1, 1): 1, (2, 2): 2, (0, 1): 3, (1, 2): 4, (0, 2): 5}
    for a in range(3):
        e = np.zeros(3)
        e[a] = 1.0
        Ah = normal_jacobian(lam, mu, rho, e)
        for b in range(3):
            r = np.zeros(9)
            r[6 + b] = 1.0
            if a == b:
                c = cp
                r[voigt[(a, a)]] = -rho * cp
                for k in range(3):
                    if k != a:
                        r[voigt[(k, k)]] = -lam / cp
            else:
                c = cs
                r[voigt[tuple(sorted((a, b)))]] = -rho * cs
            np.testing.assert_allclose(Ah @ r, c * r, rtol=1e-12, atol=1e-9)


def test_acoustic_embedding_pressure_wave():
    """mu = 0: s = -p I, p_t + K div v = 0, rho v_t + grad p = 0 (Sec. 3, acoustics)."""
    rho, K = 1000.0, 2.25e9
    c = np.sqrt(K / rho)
    Jx = jacobians(K, 0.0, rho)[0]
    # p = Z f, v_x = f travelling in +x: state (-p,-p,-p,0,0,0,1,0,0)
    r = np.array([-rho * c] * 3 + [0, 0, 0, 1, 0, 0])
    np.testing.assert_allclose(Jx @ r, c * r, rtol=1e-12)


def test_closed_form_equals_the_definition_inside_and_is_exact_at_vertices():
    """eval_basis_closed equals the collapsed-coordinate definition at interior
    points, and at the vertices and edge midpoints (where the collapsed
    coordinates are singular) it reproduces a projected polynomial exactly."""
    from oracle import basis as bas
    rng = np.random.default_rng(2)
    for N in range(1, 7):
        p = rng.dirichlet(np.ones(4), size=30)[:, 1:]
        np.testing.assert_allclose(bas.eval_basis_closed(N, p), bas.eval_basis(N, p), rtol=1e-11, atol=1e-11)
    N = 4
    q, w = quadrature.tet_rule(N + 2)
    coef = rng.standard_normal(len(bas.basis_indices(N)))
    mono = [(a, b, c) for a in range(N + 1) for b in range(N + 1) for c in range(N + 1) if a + b + c <= N]
    mc = rng.standard_normal(len(mono))
    f = lambda x: sum(m * x[:, 0] ** a * x[:, 1] ** b * x[:, 2] ** c for m, (a, b, c) in zip(mc, mono))
    dofs = (w[:, None] * bas.eval_basis(N, q) * f(q)[:, None]).sum(axis=0)
    special = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [0.5, 0.5, 0], [0, 0.5, 0.5], [0.5, 0, 0.5],
                        [0, 0, 0.5], [0, 0.3, 0.7]])
    np.testing.assert_allclose(bas.eval_basis_closed(N, special) @ dofs, f(special), rtol=1e-10, atol=1e-10)
