"""One launch per phase per sub-step (options.fused) against one launch per cluster.

In sub-step s of a macro step the clusters due are 0..k (k the largest c with
2^c dividing s, or s + 1 for the correctors, Sec. 4.4), one contiguous
element range, so the fused schedule covers them with one predictor, one
fix-up, one gravity, one second-half copy and one corrector launch. With the
same kernel choice for every element (plain kernels, or the matrix cores
with mc_min 0) the per-element arithmetic is the same as in the per-cluster
schedule, so the results must agree bit for bit, in eager launches and in
hipGraph replays. The launch counts follow the schedule: 2^(C-1) predictor
launches per macro step fused, sum_c 2^(C-1-c) per cluster.
"""
import sys

import numpy as np
import pytest

from paper_2107_06640_amd import inputs

pytestmark = pytest.mark.gpu

ZN = np.array([0.0, 0.5, 0.75, 0.875, 0.9375, 0.96875, 1.0]) * 1000.0 - 1000.0


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def lts_box():
    return inputs.coupled_box(4, 4, 6, cell=500.0, water_layers=1, z_nodes=ZN, jitter=0.1, seed=2)


@pytest.mark.parametrize("precision,kernel", [("fp64", "plain"), ("fp32", "tuned"), ("bf16", "tuned")])
def test_fused_equals_per_cluster(precision, kernel):
    from paper_2107_06640_amd import seis
    mesh, mats = lts_box()
    kw = dict(precision=precision, kernel=kernel, max_clusters=4, mc_min=0)
    runs = {}
    for name, extra in (("per-cluster", dict(fused=False)), ("fused", dict(fused=True)),
                        ("fused-graph", dict(fused=True, graph=True))):
        s = seis.from_mesh(mesh, mats, 6, **kw, **extra)
        try:
            assert s.info()["n_clusters"] == 4 and s.info()["fused"] == int(extra["fused"])
            q = inputs.random_dofs(mesh.n_elements, s.B, seed=8, acoustic=mats[2] == 0)
            eta = np.random.default_rng(9).standard_normal((s.n_gravity_faces, s.nq)) * 0.1
            s.write(q, eta)
            out = []
            for _ in range(3):
                s.step()
                out.append(s.read())
            runs[name] = out
        finally:
            s.close()
    say(f"case: fused vs per-cluster {precision}/{kernel}")
    for name in ("fused", "fused-graph"):
        for k, ((d0, e0), (d1, e1)) in enumerate(zip(runs["per-cluster"], runs[name])):
            if not np.array_equal(d0, d1):
                diff = np.abs(d0 - d1).max(axis=(1, 2)) / np.abs(d0).max()
                bad = np.nonzero(diff)[0]
                say(f"  {name} step {k}: {bad.size} elements differ, max rel {diff.max():.2e}, first {bad[:10]}")
            assert np.array_equal(d0, d1), f"{name}: macro step {k} DOFs differ"
            assert np.array_equal(e0, e1), f"{name}: macro step {k} eta differs"


@pytest.mark.parametrize("fused,expect", [(True, (8, 8)), (False, (15, 15))])
def test_launch_counts(fused, expect):
    from paper_2107_06640_amd import seis
    mesh, mats = lts_box()
    s = seis.from_mesh(mesh, mats, 5, precision="fp32", kernel="tuned", max_clusters=4, mc_min=0, fused=fused)
    try:
        s.write(inputs.random_dofs(mesh.n_elements, s.B, seed=1, acoustic=mats[2] == 0))
        s.profile(True)
        s.run(2)
        prof = s.profile_read()
        s.profile(False)
    finally:
        s.close()
    say(f"case: launch counts fused={fused}: {prof}")
    assert prof["predict"][1] == 2 * expect[0]
    assert prof["correct"][1] == 2 * expect[1]
    # every element is updated 2^(C-1-c) times per macro step either way
    assert prof["predict"][2] == 2 * (102 * 8 + 175 * 4 + 205 * 2 + 94)
