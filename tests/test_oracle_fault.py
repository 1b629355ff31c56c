"""Pins of the oracle's dynamic-rupture faces (Sec. 3, fault boundary condition).

* A locked fault (infinite cohesion) is a welded interface: the same mesh
  with ordinary interior faces gives the same state to round-off. The fault
  path evaluates both traces at the lattice points and Gauss points in time
  and interpolates its nodal flux, the interior path integrates time-
  integrated traces at quadrature points, so this checks the middle state,
  the time rule and the face integration together.
* An instantaneous stress drop on a planar fault between equal half-spaces
  radiates plane S waves; the traction balance on the fault then gives the
  slip rate 2 (tau0 - tau_S) / (rho c_s), parallel to the prestress (closed
  form). From a state at rest it holds exactly over the first step, and the
  slip follows V t afterwards up to the discretisation of the step front.
* Linear slip weakening on that fault: dS/dt = 2 (tau0 - s f(S)) / Z is linear
  in the slip S while S < D_c, so S(t) = A/k (exp(k t) - 1) (closed form).
* Under tension without cohesion the fault carries no shear traction.
* Clusters: across a fault face the two sides share a cluster; the
  assignment equals min_J (raw c_J + d(K, J)) with fault faces at distance 0
  (brute force).
* Rate-and-state friction (fast velocity weakening): the law's textbook
  limits (steady state, low-velocity logarithmic law, the weakened f_w); a
  fault started at steady-state sliding keeps sliding at that rate with its
  state unchanged over the first step; on the planar fault the slip follows
  the one-variable ODE of radiation damping, integrated with DOP853.
"""
import numpy as np
import pytest

from oracle.mesh import adjacency
from oracle.solver import assign_clusters
from paper_2107_06640_amd import inputs
from tests.parity_util import oracle_for

RHO, CS = 2700.0, 3464.0
Z = RHO * CS


def planar(nz=6):
    return inputs.fault_box(2, 2, nz, cell=1000.0, k_fault=nz // 2)


@pytest.mark.parametrize("order", [3, 4])
def test_locked_fault_is_a_welded_interface(order):
    mesh, mats = inputs.fault_box(3, 3, 4, cell=1000.0, k_fault=2, jitter=0.1, seed=1)
    assert (mesh.face_kind == inputs.FACE_FAULT).sum() == 2 * 18
    o = oracle_for(mesh, mats, order)
    q = inputs.random_dofs(mesh.n_elements, o.B, seed=3)
    o.Q[:] = q
    o.run(3)
    fk = mesh.face_kind.copy()
    fk[fk == inputs.FACE_FAULT] = inputs.FACE_INTERIOR
    welded = inputs.Mesh(xyz=mesh.xyz, tet=mesh.tet, face_kind=fk, period=mesh.period)
    o2 = oracle_for(welded, mats, order)
    o2.Q[:] = q
    o2.run(3)
    assert np.abs(o.Q - o2.Q).max() <= 1e-12 * np.abs(o2.Q).max()
    assert np.all(o.fault_rate == 0.0) and np.all(o.fault_slip == 0.0)


def test_stress_drop_slip_rate_first_step():
    mesh, mats = planar()
    o = oracle_for(mesh, mats, 3)
    tau0 = np.array([24e6, 32e6, 0.0])  # |tau0| = 40 MPa, strength 0.6 x 50 MPa = 30 MPa
    o.set_fault([-50e6, *tau0, 0.6, 0.6, 1.0, 0.0])
    o.run(1)
    V = 2.0 * (40e6 - 30e6) / Z * tau0 / 40e6
    assert np.abs(o.fault_rate - V).max() <= 1e-12 * np.abs(V).max()
    assert np.abs(o.fault_slip - V * o.time).max() <= 1e-12 * np.abs(V).max() * o.time
    # the total shear traction sits at the strength, along the prestress
    assert np.abs(o.fault_traction - 30e6 * tau0 / 40e6).max() <= 1e-6


def test_stress_drop_slip_grows_as_v_t():
    mesh, mats = planar()
    o = oracle_for(mesh, mats, 3)
    o.set_fault([-50e6, 40e6, 0.0, 0.0, 0.6, 0.6, 1.0, 0.0])
    while o.time < 0.3:  # S waves reach the absorbing ends after 0.87 s
        o.run(1)
    V = 2.0 * 10e6 / Z
    slip = o.fault_slip[..., 0]
    assert abs(slip.mean() / (V * o.time) - 1.0) < 0.01
    assert np.abs(slip / (V * o.time) - 1.0).max() < 0.03
    assert np.abs(o.fault_slip[..., 1:]).max() < 0.01 * V * o.time


def test_slip_weakening_exponential_growth():
    mesh, mats = planar()
    sig, mus, mud, dc, tau0 = 50e6, 0.6, 0.5, 0.2, 31e6
    o = oracle_for(mesh, mats, 3)
    o.set_fault([-sig, tau0, 0.0, 0.0, mus, mud, dc, 0.0])
    A, k = 2.0 * (tau0 - sig * mus) / Z, 2.0 * sig * (mus - mud) / (Z * dc)
    checked = 0
    while o.time < 0.3:
        o.run(1)
        want = A / k * (np.exp(k * o.time) - 1.0)
        if o.time > 0.1:
            assert abs(o.fault_psi.mean() / want - 1.0) < 0.05
            checked += 1
        assert want < dc
    assert checked > 10


def test_tension_without_cohesion_carries_no_shear():
    mesh, mats = planar()
    o = oracle_for(mesh, mats, 3)
    o.set_fault([10e6, 5e6, -3e6, 0.0, 0.6, 0.6, 1.0, 0.0])
    o.run(4)
    assert np.abs(o.fault_traction).max() <= 1e-6
    assert np.abs(o.fault_rate).max() > 0.0


def test_fault_faces_tie_clusters():
    mesh, _ = inputs.fault_box(3, 3, 4, cell=1.0, k_fault=2, jitter=0.1, seed=4)
    nb, _, _ = adjacency(mesh.tet, mesh.face_kind, mesh.xyz, mesh.period)
    tied = mesh.face_kind == inputs.FACE_FAULT
    E = mesh.n_elements
    rng = np.random.default_rng(6)
    dt = 2.0 ** rng.uniform(0.0, 4.0, E)
    # brute force: Floyd-Warshall with weight 0 across fault faces, 1 elsewhere
    d = np.full((E, E), 10 ** 6, dtype=np.int64)
    np.fill_diagonal(d, 0)
    for e in range(E):
        for f in range(4):
            j = nb[e, f]
            if j >= 0:
                d[e, j] = min(d[e, j], 0 if tied[e, f] else 1)
    for k in range(E):
        d = np.minimum(d, d[:, k:k + 1] + d[k:k + 1, :])
    for C in (2, 4):
        c, _ = assign_clusters(dt, nb, C, tied=tied)
        raw = np.clip(np.floor(np.log2(dt / dt.min())).astype(np.int64), 0, C - 1)
        assert np.array_equal(c, (raw[None, :] + d).min(axis=1))
        e, f = np.nonzero(tied)
        assert np.all(c[e] == c[nb[e, f]])


def test_fault_face_must_meet_a_fault_face():
    mesh, _ = inputs.fault_box(2, 2, 4, cell=1.0, k_fault=2)
    fk = mesh.face_kind.copy()
    e, f = np.argwhere(fk == inputs.FACE_FAULT)[0]
    fk[e, f] = inputs.FACE_INTERIOR
    with pytest.raises(ValueError):
        adjacency(mesh.tet, fk, mesh.xyz, mesh.period)


# ---------------------------------------------------------------------------
# rate-and-state friction (fast velocity weakening)
RS = dict(a=0.01, b=0.014, L=0.2, V0=1e-6, f0=0.6, fw=0.2, Vw=0.1)


def test_rate_state_law_textbook_limits():
    """f(V, psi_ss(V)) = f_ss(V); f_ss -> f0 - (b - a) ln(V/V0) for V << V_w and -> f_w for V >> V_w;
    for V/V0 exp(psi/a) >> 1 the regularised law is the classic a ln(V/V0) + psi."""
    from oracle.fault import rs_friction, rs_steady_state
    p = RS
    V = np.logspace(-12, 2, 29)
    pss = rs_steady_state(V, p["a"], p["b"], p["V0"], p["f0"], p["fw"], p["Vw"])
    f = rs_friction(V, pss, p["a"], p["V0"])
    fLV = p["f0"] - (p["b"] - p["a"]) * np.log(V / p["V0"])
    fss = p["fw"] + (fLV - p["fw"]) / (1.0 + (V / p["Vw"]) ** 8) ** 0.125
    assert np.allclose(f, fss, rtol=1e-12, atol=1e-14)
    slow = V < 1e-4
    assert np.allclose(f[slow], fLV[slow], rtol=1e-9)
    assert abs(f[-1] - p["fw"]) < 1e-3
    psi = 0.55
    Vb = np.array([1e-3, 1e-1, 1.0])
    assert np.allclose(rs_friction(Vb, psi, p["a"], p["V0"]), p["a"] * np.log(Vb / p["V0"]) + psi, rtol=1e-9)


def rs_case(Vi, sig=50e6, tau0=30e6):
    """Background traction in equilibrium with slip rate Vi at the first step: psi0 from
    tau0 - eta Vi = sig a asinh(Vi / (2 V0) exp(psi0 / a))."""
    p = RS
    eta = Z / 2.0
    psi0 = p["a"] * np.log(2 * p["V0"] / Vi * np.sinh((tau0 - eta * Vi) / (sig * p["a"])))
    return [-sig, tau0, 0.0, 0.0, p["a"], p["b"], p["L"], p["V0"], p["f0"], p["fw"], p["Vw"], psi0]


def test_rate_state_steady_sliding_first_step():
    """State at steady state psi_ss(Vi) and background traction sig f_ss(Vi) + eta Vi (in the
    law's own terms: f_LV and the V_w cut-off written out here): from rest the fault slides at
    Vi over the whole first step and the state does not move."""
    p = RS
    Vi, sig = 0.3, 50e6
    fLV = p["f0"] - (p["b"] - p["a"]) * np.log(Vi / p["V0"])
    fss = p["fw"] + (fLV - p["fw"]) / (1.0 + (Vi / p["Vw"]) ** 8) ** 0.125
    psi0 = p["a"] * np.log(2 * p["V0"] / Vi * np.sinh(fss / p["a"]))
    tau0 = sig * fss + Z / 2.0 * Vi
    mesh, mats = planar()
    o = oracle_for(mesh, mats, 3)
    o.set_fault([-sig, tau0, 0.0, 0.0, p["a"], p["b"], p["L"], p["V0"], p["f0"], p["fw"], p["Vw"], psi0], law=1)
    o.run(1)
    assert np.abs(o.fault_rate[..., 0] / Vi - 1.0).max() < 1e-10
    assert np.abs(o.fault_rate[..., 1:]).max() < 1e-12
    assert np.abs(o.fault_psi - psi0).max() < 1e-12
    assert np.abs(o.fault_slip[..., 0] / (Vi * o.time) - 1.0).max() < 1e-10


def test_rate_state_planar_fault_against_ode():
    """The planar stress-drop problem reduces to one ODE (radiation damping tau0 - Z V / 2 at
    the fault): integrated with DOP853 it gives the slip the DG solution must follow."""
    from scipy.integrate import solve_ivp
    from oracle.fault import rs_slip_rate, rs_steady_state
    p = RS
    prm = rs_case(0.3)
    sig, tau0, psi0 = -prm[0], prm[1], prm[11]
    eta = Z / 2.0

    def vel(psi):
        return float(rs_slip_rate(np.array([tau0]), np.array([sig]), eta, np.array([psi]), p["a"], p["V0"])[0])

    def rhs(t, y):
        V = vel(y[0])
        pss = float(rs_steady_state(np.array(V), p["a"], p["b"], p["V0"], p["f0"], p["fw"], p["Vw"]))
        return [-(V / p["L"]) * (y[0] - pss), V]

    sol = solve_ivp(rhs, (0.0, 0.3), [psi0, 0.0], method="DOP853", rtol=1e-10, atol=1e-13, dense_output=True)
    mesh, mats = planar()
    o = oracle_for(mesh, mats, 4)
    o.set_fault(prm, law=1)
    checked = 0
    while o.time < 0.3:
        o.run(1)
        if o.time > 0.1:
            want = sol.sol(o.time)[1]
            assert abs(o.fault_slip[..., 0].mean() / want - 1.0) < 0.03
            checked += 1
    assert checked > 10
    assert vel(sol.sol(0.3)[0]) > 3.0  # the fault has weakened: 0.3 -> 3.9 m/s
