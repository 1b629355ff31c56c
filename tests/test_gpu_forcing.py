"""Prescribed bottom velocity (uplift history, seis_set_uplift) against the oracle.

The graded LTS box (four clusters) with its bottom faces of kind
SEIS_FACE_VELOCITY, driven by two seeded Gaussian uplift sources with rise
times shorter than the run, from rest: FP64 plain kernels within 1e-10 of
the oracle (per field and per element, and eta) after 4 macro steps; FP32
matrix-core kernels within the LTS parity bounds, with one launch per
sub-step and per cluster; a hipGraph replay of the macro step equal to the
eager run bit for bit (the forcing's clock is a device counter, so replays
advance in time). seis_write restarts the clock.
"""
import sys

import numpy as np
import pytest

from paper_2107_06640_amd import inputs
from tests.parity_util import element_errors, field_errors, oracle_for

pytestmark = pytest.mark.gpu

ZN = np.array([0.0, 0.5, 0.75, 0.875, 0.9375, 0.96875, 1.0]) * 1000.0 - 1000.0


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def box():
    return inputs.coupled_box(4, 4, 6, cell=500.0, water_layers=1, z_nodes=ZN, jitter=0.1, seed=2,
                              bottom="velocity")


def sources(dt_macro):
    # rise times of 2-3 macro steps, so that the ramp and its end both fall in the run
    return np.array([[1.2, 700.0, 900.0, 600.0, 2.5 * dt_macro],
                     [0.8, 1500.0, 1300.0, 450.0, 1.7 * dt_macro]])


_REF = {}


def oracle_run(order, steps):
    if (order, steps) not in _REF:
        mesh, mats = box()
        o = oracle_for(mesh, mats, order, max_clusters=4)
        src = sources(o.dt_min * (1 << (o.n_clusters - 1)))
        o.uplift_sources = [tuple(r) for r in src]
        o.run(steps)
        _REF[(order, steps)] = dict(Q=o.Q.copy(), eta=o.eta.copy(), src=src, cluster=o.cluster.copy())
    return _REF[(order, steps)]


def gpu_run(order, steps, **kw):
    from paper_2107_06640_amd import seis
    mesh, mats = box()
    ref = oracle_run(order, steps)
    s = seis.from_mesh(mesh, mats, order, max_clusters=4, **kw)
    try:
        assert np.array_equal(s.cluster_of(), ref["cluster"])
        s.write(np.zeros((s.E, s.B, 9)), np.zeros((s.n_gravity_faces, s.nq)))
        s.set_uplift(ref["src"])
        s.run(steps)
        d, e = s.read()
        return d, e, ref, s.info()
    finally:
        s.close()


@pytest.mark.parametrize("order", [4, 6])
def test_uplift_forcing_fp64(order):
    # the disturbance has not reached the sea surface after 4 macro steps: eta stays 0
    d, e, ref, _ = gpu_run(order, 4, precision="fp64", kernel="plain")
    fe = field_errors(d, ref["Q"])
    ee = element_errors(d, ref["Q"])
    say(f"case: uplift fp64 order {order}: field {fe.max():.2e} element {ee.max():.2e} "
        f"max |v_z| {np.abs(ref['Q'][:, 0, 8]).max():.3e}")
    assert np.abs(ref["Q"]).max() > 0
    assert fe.max() <= 1e-10 and ee.max() <= 1e-9 and np.array_equal(e, ref["eta"])


def test_uplift_reaches_the_sea_surface_fp64():
    """A shallow box (1.5 km of rock under 500 m of water, one cluster) run until
    the uplift has lifted the sea surface: DOFs and eta within 1e-10."""
    from paper_2107_06640_amd import seis
    mesh, mats = inputs.coupled_box(3, 3, 4, cell=500.0, water_layers=1, jitter=0.1, seed=4, bottom="velocity")
    o = oracle_for(mesh, mats, 4)
    src = np.array([[1.0, 700.0, 800.0, 700.0, 0.15], [0.6, 900.0, 400.0, 500.0, 0.1]])
    o.uplift_sources = [tuple(r) for r in src]
    steps = 120
    o.run(steps)
    s = seis.from_mesh(mesh, mats, 4, precision="fp64", kernel="plain")
    try:
        s.write(np.zeros((s.E, s.B, 9)), np.zeros((s.n_gravity_faces, s.nq)))
        s.set_uplift(src)
        s.run(steps)
        d, e = s.read()
        t = s.info()["time"]
    finally:
        s.close()
    fe = field_errors(d, o.Q)
    eta = np.abs(e - o.eta).max() / np.abs(o.eta).max()
    say(f"case: uplift to the surface, t = {t:.3f} s: field {fe.max():.2e} eta {eta:.2e} "
        f"max |eta| {np.abs(o.eta).max():.3e} m")
    assert abs(t - o.time) <= 1e-12 * t
    assert np.abs(o.eta).max() > 1e-5
    assert fe.max() <= 1e-10 and eta <= 1e-10


@pytest.mark.parametrize("fused", [True, False])
def test_uplift_forcing_fp32(fused):
    d, e, ref, _ = gpu_run(5, 4, precision="fp32", kernel="tuned", mc_min=0, fused=fused)
    fe = field_errors(d, ref["Q"])
    ee = element_errors(d, ref["Q"])
    say(f"case: uplift fp32 fused={fused}: field {fe.max():.2e} element {ee.max():.2e}")
    assert fe.max() <= 6e-6 and ee.max() <= 2.5e-5 and np.array_equal(e, ref["eta"])


def test_uplift_forcing_graph_replays_advance_in_time():
    from paper_2107_06640_amd import seis
    mesh, mats = box()
    ref = oracle_run(5, 4)
    outs = []
    for graph in (False, True):
        s = seis.from_mesh(mesh, mats, 5, precision="fp32", kernel="tuned", max_clusters=4, mc_min=0, graph=graph)
        try:
            steps = []
            for _ in range(2):   # seis_write restarts the clock: both runs must agree
                s.write(np.zeros((s.E, s.B, 9)), np.zeros((s.n_gravity_faces, s.nq)))
                s.set_uplift(ref["src"])
                for _ in range(4):
                    s.step()
                    steps.append(s.read()[0])
            outs.append(steps)
        finally:
            s.close()
    say("case: uplift graph vs eager")
    for k, (a, b) in enumerate(zip(*outs)):
        assert np.array_equal(a, b), f"macro step {k}"
    assert np.array_equal(outs[0][3], outs[0][7])
    assert not np.array_equal(outs[0][1], outs[0][2])
