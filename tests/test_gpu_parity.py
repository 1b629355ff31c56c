"""Parity of the HIP library (through the C ABI) with the FP64 oracle.

FP64 acceptance: per-field relative L2 error <= 1e-10 on the DOFs and on eta
(the paper does not state a tolerance; FP64 round-off over a few steps is
~1e-13, the bar leaves margin for different summation orders).
FP32 and BF16 report per-field errors against the oracle with the bounds
derived in the design notes.
"""
import math
import sys

import numpy as np
import pytest

from paper_2107_06640_amd import inputs
from tests.parity_util import field_errors, oracle_for, submesh

pytestmark = pytest.mark.gpu

TOL64 = 1e-10


def seis():
    from paper_2107_06640_amd import seis as s
    return s


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run_pair(mesh, mats, order, steps, *, precision="fp64", kernel="plain", max_clusters=1, cfl=0.35,
             g=9.81, seed=0, eta_seed=None, tile=0, mc_min=0):
    wet = mats[2] == 0
    o = oracle_for(mesh, mats, order, cfl=cfl, g=g, max_clusters=max_clusters)
    s = seis().from_mesh(mesh, mats, order, precision=precision, kernel=kernel, cfl=cfl, g=g,
                         max_clusters=max_clusters, tile=tile, mc_min=mc_min)
    say(f"case: E={mesh.n_elements} order={order} steps={steps} {precision}/{kernel} C={max_clusters} "
        f"mc_min={mc_min}")
    assert np.array_equal(s.cluster_of(), o.cluster)
    inf = s.info()
    assert abs(inf["dt_min"] - o.dt_min) <= 1e-13 * o.dt_min
    q = inputs.random_dofs(mesh.n_elements, o.B, seed=seed, acoustic=wet)
    o.Q[:] = q
    eta = None
    if o.eta.size:
        rng = np.random.default_rng(eta_seed if eta_seed is not None else seed + 1)
        eta = rng.standard_normal(o.eta.shape) * 0.1
        o.eta[:] = eta
    s.write(q, eta)
    o.run(steps)
    s.run(steps)
    d, e = s.read()
    s.close()
    return o, d, e


def check64(o, d, e, tol=TOL64):
    fe = field_errors(d, o.Q, o.geo.absdet)
    say("field errors", np.array2string(fe, precision=2))
    assert fe.max() <= tol, fe
    if o.eta.size:
        ee = np.abs(e - o.eta).max() / np.abs(o.eta).max()
        say("eta error", ee)
        assert ee <= tol


@pytest.mark.parametrize("n", [3, 6])  # 6: the full 6 x 6 x 6-cube periodic elastic cube (1296 tets)
def test_periodic_elastic_order3_fp64(n):
    mesh = inputs.cfg1_mesh(n)
    mats = inputs.uniform_materials(mesh, 2700.0, 6000.0, 3464.0)
    o, d, e = run_pair(mesh, mats, 3, 4, cfl=0.5)
    check64(o, d, e)


def test_boundary_kinds_jittered_fp64():
    mesh = inputs.box_mesh(3, 2, 2, lengths=(3.0, 2.0, 2.0), jitter=0.2, seed=3,
                           sides={"x-": "absorbing", "x+": "wall", "y-": "free", "y+": "free",
                                  "z-": "absorbing", "z+": "wall"})
    mats = inputs.uniform_materials(mesh, 2500.0, 5000.0, 2800.0)
    o, d, e = run_pair(mesh, mats, 4, 3)
    check64(o, d, e)


@pytest.mark.parametrize("order", [3, 4, 5, 6, 7])
def test_coupled_gravity_all_orders_fp64(order):
    mesh, mats = inputs.coupled_box(3, 2, 4, cell=500.0, water_layers=2, jitter=0.15, seed=order)
    o, d, e = run_pair(mesh, mats, order, 2, seed=order)
    check64(o, d, e)


def test_lts_three_clusters_fp64():
    zn = np.array([0.0, 0.6, 0.85, 0.95, 1.0]) * 1000.0 - 1000.0
    mesh, mats = inputs.coupled_box(2, 2, 4, cell=500.0, water_layers=1, z_nodes=zn)
    o, d, e = run_pair(mesh, mats, 4, 2, max_clusters=3)
    assert o.n_clusters >= 2
    check64(o, d, e)


def test_lts_graded_elastic_fp64():
    mesh = inputs.box_mesh(2, 2, 4, z_nodes=[0.0, 0.6, 0.85, 0.95, 1.0])
    mats = inputs.uniform_materials(mesh, 2700.0, 6000.0, 3464.0)
    o, d, e = run_pair(mesh, mats, 3, 2, max_clusters=3, cfl=0.5)
    assert o.n_clusters == 3
    check64(o, d, e)


def test_fp32_plain_coupled():
    mesh, mats = inputs.coupled_box(3, 2, 4, cell=500.0, water_layers=2, jitter=0.15, seed=5)
    o, d, e = run_pair(mesh, mats, 5, 3, precision="fp32")
    fe = field_errors(d, o.Q, o.geo.absdet)
    say("fp32 field errors", np.array2string(fe, precision=2))
    assert fe.max() < 1e-4


def test_schedule_order_errors():
    zn = np.array([0.0, 0.6, 0.85, 0.95, 1.0])
    mesh = inputs.box_mesh(2, 2, 4, z_nodes=zn)
    mats = inputs.uniform_materials(mesh, 2700.0, 6000.0, 3464.0)
    s = seis().from_mesh(mesh, mats, 3, kernel="plain", max_clusters=3, cfl=0.5)
    S = seis()
    with pytest.raises(S.SeisError) as ex:
        s.correct(0)
    assert ex.value.code == -4
    with pytest.raises(S.SeisError) as ex:
        s.predict(7)
    assert ex.value.code == -5
    s.predict(0)
    with pytest.raises(S.SeisError):
        s.predict(0)
    with pytest.raises(S.SeisError):
        s.read()
    s.predict(1)
    s.predict(2)
    s.correct(0)
    s.close()


def test_fp64_is_deterministic():
    mesh, mats = inputs.coupled_box(3, 2, 4, cell=500.0, water_layers=2, jitter=0.15, seed=1)
    q = inputs.random_dofs(mesh.n_elements, 35, seed=4, acoustic=mats[2] == 0)
    outs = []
    for _ in range(2):
        s = seis().from_mesh(mesh, mats, 5, kernel="plain")
        s.write(q)
        s.run(3)
        outs.append(s.read())
        s.close()
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def test_invalid_inputs_return_errors():
    S = seis()
    mesh, mats = inputs.coupled_box(2, 2, 2, cell=500.0, water_layers=1)
    rho, lam, mu = mats
    with pytest.raises(S.SeisError) as ex:
        S.from_mesh(mesh, (rho, lam, np.full_like(mu, 1e9)), 4)   # gravity face on elastic elements
    assert ex.value.code == -1
    with pytest.raises(S.SeisError):
        S.from_mesh(mesh, mats, 9)
    bad = inputs.Mesh(mesh.xyz.copy(), mesh.tet.copy(), mesh.face_kind.copy(), mesh.period.copy())
    bad.tet[0, 1] = bad.tet[0, 0]
    with pytest.raises(S.SeisError):
        S.from_mesh(bad, mats, 4)


# ---------------------------------------------------------------------------
# Tuned (matrix-core) kernels. FP32 operands: per-field relative L2 against the
# FP64 oracle below 2e-5 over a few steps (FP32 round-off ~6e-8 per operation,
# amplified by the CK chain and the Lagrange lift). BF16 operands: below 3e-2
# (operand round-off 2^-9 per value; the state stays FP32).
TOL32 = 2e-5
TOL16 = 3e-2


@pytest.mark.parametrize("order", [3, 4, 5, 6, 7])
def test_tuned_fp32_coupled_gravity(order):
    mesh, mats = inputs.coupled_box(4, 3, 4, cell=500.0, water_layers=2, jitter=0.15, seed=order)
    o, d, e = run_pair(mesh, mats, order, 2, precision="fp32", kernel="tuned", seed=order)
    fe = field_errors(d, o.Q, o.geo.absdet)
    ee = np.abs(e - o.eta).max() / np.abs(o.eta).max()
    say("tuned fp32 field errors", np.array2string(fe, precision=2), "eta", ee)
    assert fe.max() < TOL32 and ee < TOL32


def test_tuned_fp32_boundary_kinds_and_ragged_groups():
    # 3*2*3*6 = 108 elements: 6 full 16-element groups and a ragged tail of 12
    mesh = inputs.box_mesh(3, 2, 3, lengths=(3.0, 2.0, 3.0), jitter=0.2, seed=4,
                           sides={"x-": "absorbing", "x+": "wall", "y-": "free", "y+": "free",
                                  "z-": "absorbing", "z+": "wall"})
    mats = inputs.uniform_materials(mesh, 2500.0, 5000.0, 2800.0)
    o, d, e = run_pair(mesh, mats, 5, 3, precision="fp32", kernel="tuned")
    fe = field_errors(d, o.Q, o.geo.absdet)
    say("tuned fp32 boundary field errors", np.array2string(fe, precision=2))
    assert fe.max() < TOL32


def test_tuned_fp32_lts():
    zn = np.array([0.0, 0.6, 0.85, 0.95, 1.0]) * 1000.0 - 1000.0
    mesh, mats = inputs.coupled_box(4, 4, 4, cell=500.0, water_layers=1, z_nodes=zn)
    o, d, e = run_pair(mesh, mats, 5, 2, precision="fp32", kernel="tuned", max_clusters=3)
    assert o.n_clusters >= 2
    fe = field_errors(d, o.Q, o.geo.absdet)
    say("tuned fp32 lts field errors", np.array2string(fe, precision=2))
    assert fe.max() < TOL32


@pytest.mark.parametrize("order", [3, 4, 5, 6, 7])
def test_tuned_bf16_coupled_gravity(order):
    mesh, mats = inputs.coupled_box(4, 3, 4, cell=500.0, water_layers=2, jitter=0.15, seed=order)
    o, d, e = run_pair(mesh, mats, order, 2, precision="bf16", kernel="tuned", seed=order)
    fe = field_errors(d, o.Q, o.geo.absdet)
    ee = np.abs(e - o.eta).max() / np.abs(o.eta).max()
    say("tuned bf16 field errors", np.array2string(fe, precision=2), "eta", ee)
    assert fe.max() < TOL16 and ee < TOL16


@pytest.mark.parametrize("tile", [16, 32, 64])
def test_tuned_tiles_agree(tile):
    mesh, mats = inputs.coupled_box(4, 3, 4, cell=500.0, water_layers=2, jitter=0.15, seed=9)
    o, d, e = run_pair(mesh, mats, 4, 1, precision="fp32", kernel="tuned", tile=tile, seed=9)
    assert field_errors(d, o.Q, o.geo.absdet).max() < TOL32


@pytest.mark.parametrize("mc_min", [0, 160])
@pytest.mark.parametrize("precision,tol", [("fp32", TOL32), ("bf16", TOL16)])
def test_tuned_lts_interfaces_with_gravity(precision, tol, mc_min):
    # three clusters (137, 185 and 158 elements) over a graded water column
    # with a gravity surface. mc_min 0: the matrix-core kernels run every
    # element, including those handing over to finer (half-step traces) and
    # coarser (accumulated halves) neighbours. mc_min 160: the middle cluster
    # runs on the matrix cores and its finer and coarser neighbours on the
    # plain kernels, so every hand-over crosses between the two kernel kinds.
    zn = np.array([0.0, 0.5, 0.75, 0.875, 0.9375, 1.0]) * 1000.0 - 1000.0
    mesh, mats = inputs.coupled_box(4, 4, 5, cell=500.0, water_layers=1, z_nodes=zn, jitter=0.1, seed=2)
    o, d, e = run_pair(mesh, mats, 5, 2, precision=precision, kernel="tuned", max_clusters=4, seed=6,
                       mc_min=mc_min)
    assert list(np.bincount(o.cluster)) == [137, 185, 158]
    fe = field_errors(d, o.Q, o.geo.absdet)
    ee = np.abs(e - o.eta).max() / np.abs(o.eta).max()
    say(f"tuned {precision} lts+gravity field errors", np.array2string(fe, precision=3), "eta", ee)
    assert fe.max() < tol and ee < tol
