"""Orders 2 and 8 (degrees 1 and 7) on the plain kernels, against the oracle.

The matrix-core kernels cover orders 3-7; the plain kernels (one work-group
per element) take the whole range 2-8 of the method (Sec. 4.1 places no
bound on the degree). Parity bars as in the other FP64 tests: per-field
relative L2 <= 1e-10 on the state and eta, per element <= 1e-9; FP32 plain
kernels within 1e-4 per field after 3 steps. Order 2 with a dynamic-rupture
fault (part of it slipping) at the fault bars of the fault tests. Set-up
rejects the matrix-core kernels outside 3-7 and fault faces at order 8 with
a message that names the range.
"""
import sys

import numpy as np
import pytest

from paper_2107_06640_amd import inputs
from tests.parity_util import element_errors, field_errors, oracle_for

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run_pair(mesh, mats, order, steps, *, precision="fp64", max_clusters=1, cfl=0.35, seed=0):
    from paper_2107_06640_amd import seis
    wet = mats[2] == 0
    o = oracle_for(mesh, mats, order, cfl=cfl, g=9.81, max_clusters=max_clusters)
    s = seis.from_mesh(mesh, mats, order, precision=precision, kernel="plain", cfl=cfl, g=9.81,
                       max_clusters=max_clusters)
    try:
        say(f"case: E={mesh.n_elements} order={order} steps={steps} {precision}/plain clusters={o.n_clusters}")
        assert np.array_equal(s.cluster_of(), o.cluster)
        assert s.info()["n_basis"] == o.B
        q = inputs.random_dofs(mesh.n_elements, o.B, seed=seed, acoustic=wet)
        o.Q[:] = q
        eta = None
        if o.eta.size:
            eta = np.random.default_rng(seed + 1).standard_normal(o.eta.shape) * 0.1
            o.eta[:] = eta
        s.write(q, eta)
        o.run(steps)
        s.run(steps)
        d, e = s.read()
    finally:
        s.close()
    fe = field_errors(d, o.Q, o.geo.absdet)
    ee = element_errors(d, o.Q)
    eta_err = float(np.abs(e - o.eta).max() / np.abs(o.eta).max()) if o.eta.size else 0.0
    say(f"  field {fe.max():.2e} element {ee.max():.2e} eta {eta_err:.2e}")
    return fe, ee, eta_err


@pytest.mark.parametrize("order", [2, 8])
def test_periodic_elastic_fp64(order):
    mesh = inputs.cfg1_mesh(3)
    mats = inputs.uniform_materials(mesh, 2700.0, 6000.0, 3464.0)
    fe, ee, _ = run_pair(mesh, mats, order, 3, cfl=0.5, seed=order)
    assert fe.max() <= 1e-10 and ee.max() <= 1e-9


@pytest.mark.parametrize("order", [2, 8])
def test_coupled_gravity_fp64(order):
    mesh, mats = inputs.coupled_box(3, 2, 4, cell=500.0, water_layers=2, jitter=0.15, seed=order)
    fe, ee, eta_err = run_pair(mesh, mats, order, 2, seed=order)
    assert fe.max() <= 1e-10 and ee.max() <= 1e-9 and eta_err <= 1e-10


@pytest.mark.parametrize("order", [2, 8])
def test_lts_fp64(order):
    zn = np.array([0.0, 0.6, 0.85, 0.95, 1.0]) * 1000.0 - 1000.0
    mesh, mats = inputs.coupled_box(2, 2, 4, cell=500.0, water_layers=1, z_nodes=zn)
    fe, ee, eta_err = run_pair(mesh, mats, order, 2, max_clusters=3, seed=order + 10)
    assert fe.max() <= 1e-10 and ee.max() <= 1e-9 and eta_err <= 1e-10


@pytest.mark.parametrize("order", [2, 8])
def test_coupled_gravity_fp32_plain(order):
    mesh, mats = inputs.coupled_box(3, 2, 4, cell=500.0, water_layers=2, jitter=0.15, seed=order + 20)
    fe, _, eta_err = run_pair(mesh, mats, order, 3, precision="fp32", seed=order + 20)
    assert fe.max() < 1e-4 and eta_err < 1e-4


def test_fault_order2_fp64():
    from tests.test_gpu_fault import TOL, check, gpu_run, jittered_box, oracle_result
    ref = oracle_result("jit", jittered_box, 2, 4, 1)
    say("case: jittered fault order=2 fp64/plain 4 steps")
    d, flt = gpu_run(jittered_box, 2, 4, ref, precision="fp64", kernel="plain", mc_min=0)
    check(d, flt, ref, TOL["fp64"])


def test_out_of_range_rejected():
    from paper_2107_06640_amd import seis
    mesh, mats = inputs.coupled_box(2, 2, 2, cell=500.0, water_layers=1)
    for order, kw, text in [(2, dict(kernel="tuned", precision="fp32"), "3..7"),
                            (8, dict(kernel="tuned", precision="bf16"), "3..7"),
                            (1, dict(kernel="plain"), "2..8"), (9, dict(kernel="plain"), "2..8"),
                            (7, dict(kernel="tuned", precision="bf16x3"), "3..6")]:
        with pytest.raises(Exception, match=text.replace(".", r"\.")):
            seis.from_mesh(mesh, mats, order, **kw)
    fmesh, fmats = inputs.fault_box(2, 2, 2, cell=1000.0, k_fault=1)
    with pytest.raises(Exception, match=r"2\.\.7"):
        seis.from_mesh(fmesh, fmats, 8, kernel="plain")
