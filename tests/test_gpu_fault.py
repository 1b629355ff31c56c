"""Dynamic-rupture faces on the GPU against the oracle and closed forms.

The friction kernel (FP64 arithmetic) reads both sides' stored time
derivatives, applies the slip-weakening law at the face nodes and Gauss
points in time, and hands each side its time-averaged middle state (Sec. 3,
fault boundary condition; Sec. 4.2, middle state).

Cases:
* A jittered (non-planar) fault between rock layers, a small seeded random
  state, a background traction of 20 MPa against a static strength of
  30 MPa except on a central nucleation patch at 31 MPa, so that part of the
  fault slips (and weakens past D_c) and part stays locked: against the
  oracle after 4 steps, the
  element state per field and per element, and the fault's slip, slip path,
  slip rate and tractions point by point (matched by coordinates). FP64
  plain at 1e-10 (state) and 1e-9 (fault); FP32 matrix-core kernels at the
  FP32 bars of the other parity tests.
* The same with rate-2 LTS: graded layers give two clusters, with fault
  faces in both (the two sides of a fault face share a cluster).
* A planar fault under an instantaneous stress drop, from rest: the slip
  rate over the first step is 2 (tau0 - tau_S) / (rho c_s) at every point,
  parallel to the prestress (closed form), and the slip after 0.3 s is V t
  to 1%.
* A graph-replayed macro step gives the eager result bit for bit, and
  seis_write puts the fault back at rest.
"""
import sys

import numpy as np
import pytest

from paper_2107_06640_amd import inputs
from tests.parity_util import element_errors, field_errors, oracle_for

pytestmark = pytest.mark.gpu

RHO, CS = 2700.0, 3464.0
TOL = {"fp64": dict(field=1e-10, elem=1e-9, fault=1e-9), "fp32": dict(field=6e-6, elem=2.5e-5, fault=2e-4)}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def jittered_box():
    return inputs.fault_box(3, 3, 4, cell=1000.0, k_fault=2, jitter=0.1, seed=1)


def graded_box():
    zn = np.array([0.0, 600.0, 1100.0, 1500.0, 1800.0, 2000.0, 2150.0]) - 1100.0
    return inputs.fault_box(3, 3, 6, cell=700.0, k_fault=2, jitter=0.1, seed=3, z_nodes=zn)


def fault_table(o):
    """Oracle fault state as rows (x, y, z, slip 3, psi, V 3, T 3, S), one per point."""
    return np.concatenate([o.fault_points.reshape(-1, 3), o.fault_slip.reshape(-1, 3),
                           o.fault_psi.reshape(-1, 1), o.fault_rate.reshape(-1, 3),
                           o.fault_traction.reshape(-1, 3), o.fault_normal.reshape(-1, 1)], axis=1)


def fault_params(o):
    """Per face: s0 = -50 MPa, mu_s 0.6, mu_d 0.5, D_c 2 mm; tau0 = 31 MPa along x within
    1 km of the box's vertical axis (the face centroid), else (20, 3) MPa."""
    c = o.fault_points.mean(axis=1)
    mid = 0.5 * (o.geo.xyz.min(axis=0) + o.geo.xyz.max(axis=0))
    P = np.tile([-50e6, 20e6, 3e6, 0.0, 0.6, 0.5, 0.002, 0.0], (c.shape[0], 1))
    P[np.hypot(c[:, 0] - mid[0], c[:, 1] - mid[1]) < 1000.0, 1:3] = (31e6, 0.0)
    return P


def match(gpu, ref):
    """gpu rows [F, nf, 14] reordered to the reference rows [F * nf, 14].

    Both list the faces in the same order (by '-' element, local face); the
    points of a face are matched by their coordinates (points on shared edges
    of neighbouring faces coincide, so the matching is per face).
    """
    F, nf = gpu.shape[:2]
    r = ref.reshape(F, nf, -1)
    d = ((gpu[:, None, :, :3] - r[:, :, None, :3]) ** 2).sum(axis=3)      # [F, ref point, gpu point]
    idx = d.argmin(axis=2)
    assert np.sqrt(np.take_along_axis(d, idx[..., None], 2)).max() < 1e-6 * np.abs(ref[:, :3]).max()
    assert all(np.unique(idx[f]).size == nf for f in range(F))
    return np.take_along_axis(gpu, idx[..., None], 1).reshape(F * nf, -1)


_ORACLE = {}


def oracle_result(name, build, order, steps, max_clusters):
    key = (name, order, steps, max_clusters)
    if key not in _ORACLE:
        mesh, mats = build()
        o = oracle_for(mesh, mats, order, max_clusters=max_clusters)
        P = fault_params(o)
        o.set_fault(P)
        q = inputs.random_dofs(mesh.n_elements, o.B, seed=order + 40, stress_scale=1e4, velocity_scale=1e4 / 3e6)
        o.Q[:] = q
        o.run(steps)
        _ORACLE[key] = dict(q0=q, Q=o.Q.copy(), fault=fault_table(o), cluster=o.cluster.copy(), params=P)
    return _ORACLE[key]


def gpu_run(build, order, steps, ref, **kw):
    from paper_2107_06640_amd import seis
    mesh, mats = build()
    s = seis.from_mesh(mesh, mats, order, **kw)
    try:
        assert np.array_equal(s.cluster_of(), ref["cluster"])
        assert s.info()["n_fault_faces"] == ref["fault"].shape[0] // s.info()["n_face_nodes"]
        s.set_fault(ref["params"])
        s.write(ref["q0"])
        s.run(steps)
        d, _ = s.read()
        return d, s.fault_read()
    finally:
        s.close()


def check(d, flt, ref, tol):
    fe = field_errors(d, ref["Q"])
    ee = element_errors(d, ref["Q"])
    g = match(flt, ref["fault"])
    r = ref["fault"]
    slipping = r[:, 6] > 0
    weakened = r[:, 6] > 0.002
    errs = {}
    for name, cols in (("slip", slice(3, 6)), ("psi", slice(6, 7)), ("rate", slice(7, 10)),
                       ("traction", slice(10, 13)), ("normal", slice(13, 14))):
        errs[name] = np.abs(g[:, cols] - r[:, cols]).max() / max(np.abs(r[:, cols]).max(), 1e-300)
    say(f"  field {fe.max():.2e} element {ee.max():.2e} fault "
        + " ".join(f"{k} {v:.1e}" for k, v in errs.items())
        + f" slipping points {int(slipping.sum())}/{slipping.size} weakened past D_c {int(weakened.sum())}")
    assert 0 < slipping.sum() < slipping.size  # part of the fault slips, part stays locked
    assert weakened.sum() > 0
    assert fe.max() <= tol["field"] and ee.max() <= tol["elem"]
    assert max(errs.values()) <= tol["fault"]


@pytest.mark.parametrize("precision,kernel", [("fp64", "plain"), ("fp32", "tuned")])
@pytest.mark.parametrize("order", [4, 6])
def test_fault_against_oracle(order, precision, kernel):
    ref = oracle_result("jit", jittered_box, order, 4, 1)
    say(f"case: jittered fault order={order} {precision}/{kernel} 4 steps")
    d, flt = gpu_run(jittered_box, order, 4, ref, precision=precision, kernel=kernel, mc_min=0)
    check(d, flt, ref, TOL[precision])


@pytest.mark.parametrize("precision,kernel", [("fp64", "plain"), ("fp32", "tuned")])
def test_fault_with_lts_against_oracle(precision, kernel):
    order = 5
    ref = oracle_result("lts", graded_box, order, 3, 3)
    cl = np.bincount(ref["cluster"])
    say(f"case: graded fault box order={order} {precision}/{kernel} clusters {cl.tolist()} 3 macro steps")
    assert cl.size == 2
    d, flt = gpu_run(graded_box, order, 3, ref, precision=precision, kernel=kernel, max_clusters=3, mc_min=0)
    check(d, flt, ref, TOL[precision])


@pytest.mark.parametrize("precision,kernel,tol", [("fp64", "plain", 1e-12), ("fp32", "tuned", 1e-5)])
def test_stress_drop_closed_form(precision, kernel, tol):
    from paper_2107_06640_amd import seis
    mesh, mats = inputs.fault_box(2, 2, 6, cell=1000.0, k_fault=3)
    tau0 = np.array([24e6, 32e6, 0.0])
    s = seis.from_mesh(mesh, mats, 4, precision=precision, kernel=kernel, mc_min=0)
    try:
        s.set_fault([-50e6, *tau0, 0.6, 0.6, 1.0, 0.0])
        s.write(np.zeros((mesh.n_elements, s.B, 9)))
        s.step()
        V = 2.0 * 10e6 / (RHO * CS) * tau0 / 40e6
        f = s.fault_read()
        say(f"case: stress drop {precision}/{kernel}: V {f[..., 7:10].reshape(-1, 3).mean(axis=0)} closed form {V}")
        assert np.abs(f[..., 7:10] - V).max() <= tol * np.abs(V).max()
        dt = s.info()["dt_min"]
        steps = int(round(0.3 / dt))
        s.run(steps - 1)
        f = s.fault_read()
        t = steps * dt
        ratio = f[..., 3:6].reshape(-1, 3) @ (tau0 / 40e6) / (np.linalg.norm(V) * t)
        say(f"  slip / (V t) after {t:.3f} s: {ratio.min():.4f} .. {ratio.max():.4f}")
        assert abs(ratio.mean() - 1.0) < 0.01 and np.abs(ratio - 1.0).max() < 0.03
    finally:
        s.close()


def test_graph_replay_and_write_reset():
    from paper_2107_06640_amd import seis
    mesh, mats = graded_box()
    ref = oracle_result("lts", graded_box, 5, 3, 3)
    out = []
    for graph in (False, True):
        s = seis.from_mesh(mesh, mats, 5, precision="fp32", kernel="tuned", max_clusters=3, mc_min=0, graph=graph)
        try:
            s.set_fault(ref["params"])
            q = ref["q0"]
            s.write(q)
            s.run(3)
            d, _ = s.read()
            out.append((d, s.fault_read()))
            s.write(q)
            assert np.all(s.fault_read()[..., 3:] == 0.0)
        finally:
            s.close()
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
    assert np.abs(out[0][1][..., 3:6]).max() > 0.0


# ---------------------------------------------------------------------------
# rate-and-state friction (fast velocity weakening)
RS = dict(a=0.01, b=0.014, L=0.2, V0=1e-6, f0=0.6, fw=0.2, Vw=0.1)


def rs_psi(tau, sig, V):
    """State in which background traction tau slides at V against the radiation damping eta V."""
    p = RS
    return p["a"] * np.log(2 * p["V0"] / V * np.sinh((tau - RHO * CS / 2.0 * V) / (sig * p["a"])))


def rs_params(o):
    """Per face: s0 = -50 MPa, creeping at 1e-9 m/s under 20 MPa, except a central patch at 31 MPa
    with the same state (it accelerates)."""
    p = RS
    c = o.fault_points.mean(axis=1)
    mid = 0.5 * (o.geo.xyz.min(axis=0) + o.geo.xyz.max(axis=0))
    psi0 = rs_psi(20e6, 50e6, 1e-9)
    P = np.tile([-50e6, 20e6, 0.0, 0.0, p["a"], p["b"], p["L"], p["V0"], p["f0"], p["fw"], p["Vw"], psi0],
                (c.shape[0], 1))
    P[np.hypot(c[:, 0] - mid[0], c[:, 1] - mid[1]) < 1000.0, 1] = 31e6
    return P


def rs_oracle(order, steps=4):
    key = ("rs", order, steps)
    if key not in _ORACLE:
        mesh, mats = jittered_box()
        o = oracle_for(mesh, mats, order)
        P = rs_params(o)
        o.set_fault(P, law=1)
        q = inputs.random_dofs(mesh.n_elements, o.B, seed=order + 50, stress_scale=1e4, velocity_scale=1e4 / 3e6)
        o.Q[:] = q
        o.run(steps)
        _ORACLE[key] = dict(q0=q, Q=o.Q.copy(), fault=fault_table(o), cluster=o.cluster.copy(), params=P)
    return _ORACLE[key]


@pytest.mark.parametrize("precision,kernel", [("fp64", "plain"), ("fp32", "tuned")])
@pytest.mark.parametrize("order", [4, 6])
def test_rate_state_against_oracle(order, precision, kernel):
    from paper_2107_06640_amd import seis
    ref = rs_oracle(order)
    say(f"case: rate-and-state fault order={order} {precision}/{kernel} 4 steps")
    mesh, mats = jittered_box()
    s = seis.from_mesh(mesh, mats, order, precision=precision, kernel=kernel, mc_min=0)
    try:
        s.set_fault(ref["params"], law=1)
        s.write(ref["q0"])
        s.run(4)
        d, _ = s.read()
        flt = s.fault_read()
    finally:
        s.close()
    fe = field_errors(d, ref["Q"])
    ee = element_errors(d, ref["Q"])
    g = match(flt, ref["fault"])
    r = ref["fault"]
    errs = {name: np.abs(g[:, cols] - r[:, cols]).max() / max(np.abs(r[:, cols]).max(), 1e-300)
            for name, cols in (("slip", slice(3, 6)), ("psi", slice(6, 7)), ("rate", slice(7, 10)),
                               ("traction", slice(10, 13)), ("normal", slice(13, 14)))}
    fast = np.linalg.norm(r[:, 7:10], axis=1)
    say(f"  field {fe.max():.2e} element {ee.max():.2e} fault " + " ".join(f"{k} {v:.1e}" for k, v in errs.items())
        + f" slip rate {fast.min():.2e} .. {fast.max():.2e} m/s")
    assert fast.max() > 1e3 * fast.min()  # creeping and accelerated points
    tol = TOL[precision]
    assert fe.max() <= tol["field"] and ee.max() <= tol["elem"] and max(errs.values()) <= tol["fault"]


@pytest.mark.parametrize("precision,kernel", [("fp64", "plain"), ("fp32", "tuned")])
def test_rate_state_planar_fault_against_ode(precision, kernel):
    """Planar fault: the slip follows the radiation-damping ODE (DOP853) to 3% after 0.1 s."""
    from scipy.integrate import solve_ivp
    from oracle.fault import rs_slip_rate, rs_steady_state
    from paper_2107_06640_amd import seis
    p = RS
    sig, tau0 = 50e6, 30e6
    psi0 = rs_psi(tau0, sig, 0.3)
    eta = RHO * CS / 2.0

    def vel(psi):
        return float(rs_slip_rate(np.array([tau0]), np.array([sig]), eta, np.array([psi]), p["a"], p["V0"])[0])

    def rhs(t, y):
        V = vel(y[0])
        pss = float(rs_steady_state(np.array(V), p["a"], p["b"], p["V0"], p["f0"], p["fw"], p["Vw"]))
        return [-(V / p["L"]) * (y[0] - pss), V]

    sol = solve_ivp(rhs, (0.0, 0.3), [psi0, 0.0], method="DOP853", rtol=1e-10, atol=1e-13, dense_output=True)
    mesh, mats = inputs.fault_box(2, 2, 6, cell=1000.0, k_fault=3)
    s = seis.from_mesh(mesh, mats, 4, precision=precision, kernel=kernel, mc_min=0)
    try:
        s.set_fault([-sig, tau0, 0.0, 0.0, p["a"], p["b"], p["L"], p["V0"], p["f0"], p["fw"], p["Vw"], psi0], law=1)
        s.write(np.zeros((mesh.n_elements, s.B, 9)))
        dt = s.info()["dt_min"]
        worst, n = 0.0, 0
        for k in range(1, int(0.3 / dt) + 1):
            s.step()
            if k * dt > 0.1 and k % 5 == 0:
                slip = s.fault_read()[..., 3].mean()
                worst = max(worst, abs(slip / sol.sol(k * dt)[1] - 1.0))
                n += 1
        say(f"case: rate-and-state planar fault {precision}/{kernel}: worst slip error vs ODE {worst:.2e} over {n} samples")
        assert n > 5 and worst < 0.03
    finally:
        s.close()
