"""The 4-quantity form of acoustic elements on the matrix cores.

With mu = 0 the stress of the velocity-stress system is -p I (Sec. 4.1): the
normal stresses coincide and the shear stresses vanish, so an acoustic element
needs s_xx (= -p) and the velocity only. A 16-element group whose elements
are all acoustic runs in that form (options.acoustic, the default); its face
fluxes read the neighbour's full trace, so the elastic-acoustic seafloor
(Sec. 4.2) couples the two forms. The oracle integrates the nine-quantity
embedding everywhere: for an isotropic acoustic state the two agree up to
rounding.

Mesh: the graded ocean-over-solid box of the LTS parity tests with three of
its six layers water (4 x 4 x 6 cubes x 6 = 576 tetrahedra, half of them
acoustic, spread over three LTS clusters), gravity surface on top.

Cases:
* the number of 4-quantity groups equals the count from the library's element
  order (by cluster, then cluster-interface flag, then acoustic first);
* FP32 and BF16 at orders 5, 6 and 7 against the oracle, 6 macro steps, with
  the bounds of the LTS parity tests, per field and per element;
* FP32 with and without the 4-quantity form on the same input: equal to FP32
  rounding, and the isotropy of every water element's stress kept exactly in
  at least the elements of the 4-quantity groups.
"""
import sys

import numpy as np
import pytest

from oracle.mesh import adjacency
from paper_2107_06640_amd import inputs
from tests.parity_util import element_errors, field_errors, oracle_for

pytestmark = pytest.mark.gpu

ZN = np.array([0.0, 0.5, 0.75, 0.875, 0.9375, 0.96875, 1.0]) * 1000.0 - 1000.0
STEPS = 6
TOL = {
    "fp32": dict(field=6e-6, elem=2.5e-5, eta=1.5e-6),
    "bf16": dict(field=0.1, elem=0.25, eta=0.035),
}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def wet_box():
    return inputs.coupled_box(4, 4, 6, cell=500.0, water_layers=3, z_nodes=ZN, jitter=0.1, seed=5)


def expected_groups(mesh, mats, cluster):
    """16-element groups that are all acoustic in the library's element order."""
    nb, _, _ = adjacency(mesh.tet, mesh.face_kind, mesh.xyz, mesh.period)
    E = mesh.n_elements
    iface = np.zeros(E, bool)
    for f in range(4):
        j = nb[:, f]
        iface |= (j >= 0) & (cluster[np.maximum(j, 0)] != cluster)
    elastic = mats[2] > 0
    order = np.lexsort((elastic, iface, cluster))  # stable: last key first
    wet = ~elastic[order]
    n = 0
    for g0 in range(0, E, 16):
        n += int(wet[g0:g0 + 16].all())
    return n


_ORACLE = {}


def oracle_result(order):
    if order not in _ORACLE:
        mesh, mats = wet_box()
        o = oracle_for(mesh, mats, order, max_clusters=4)
        q = inputs.random_dofs(mesh.n_elements, o.B, seed=order + 20, acoustic=mats[2] == 0)
        eta = np.random.default_rng(order + 200).standard_normal(o.eta.shape) * 0.1
        o.Q[:] = q
        o.eta[:] = eta
        o.run(STEPS)
        _ORACLE[order] = dict(q0=q, eta0=eta, Q=o.Q.copy(), eta=o.eta.copy(), cluster=o.cluster.copy())
    return _ORACLE[order]


def gpu_run(order, ref, **kw):
    from paper_2107_06640_amd import seis
    mesh, mats = wet_box()
    s = seis.from_mesh(mesh, mats, order, kernel="tuned", max_clusters=4, mc_min=0, **kw)
    try:
        assert np.array_equal(s.cluster_of(), ref["cluster"])
        inf = s.info()
        s.write(ref["q0"], ref["eta0"])
        s.run(STEPS)
        d, e = s.read()
        return d, e, inf
    finally:
        s.close()


def test_group_count_follows_element_order():
    mesh, mats = wet_box()
    ref = oracle_result(5)
    n = expected_groups(mesh, mats, ref["cluster"])
    say(f"clusters {np.bincount(ref['cluster']).tolist()} water {int((mats[2] == 0).sum())} "
        f"4-quantity groups {n}")
    assert n >= 12  # 288 water elements over three clusters
    assert len(np.unique(ref["cluster"][mats[2] == 0])) >= 2
    _, _, inf = gpu_run(5, ref, precision="fp32")
    assert inf["n_acoustic_groups"] == n
    _, _, inf0 = gpu_run(5, ref, precision="fp32", acoustic=False)
    assert inf0["n_acoustic_groups"] == 0


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
@pytest.mark.parametrize("order", [5, 6, 7])
def test_four_quantity_form_matches_oracle(order, precision):
    ref = oracle_result(order)
    say(f"case: wet box order={order} {precision}/tuned acoustic groups, {STEPS} macro steps")
    d, e, inf = gpu_run(order, ref, precision=precision)
    assert inf["n_acoustic_groups"] > 0
    fe = field_errors(d, ref["Q"])
    ee = element_errors(d, ref["Q"])
    eta = np.abs(e - ref["eta"]).max() / np.abs(ref["eta"]).max()
    say(f"  field {np.array2string(fe, precision=2)} element max {ee.max():.2e} eta {eta:.2e}")
    t = TOL[precision]
    assert fe.max() <= t["field"] and ee.max() <= t["elem"] and eta <= t["eta"]


def test_four_and_nine_quantity_forms_agree():
    mesh, mats = wet_box()
    order = 6
    ref = oracle_result(order)
    wet = mats[2] == 0
    d4, e4, inf4 = gpu_run(order, ref, precision="fp32")
    d9, e9, inf9 = gpu_run(order, ref, precision="fp32", acoustic=False)
    assert inf4["n_acoustic_groups"] > 0 and inf9["n_acoustic_groups"] == 0
    fe = field_errors(d4, d9)
    ee = element_errors(d4, d9)
    bitwise = int(np.sum(np.all(d4 == d9, axis=(1, 2))))
    say(f"  4 vs 9 quantities: field {np.array2string(fe, precision=2)} element max {ee.max():.2e} "
        f"bitwise-equal elements {bitwise}/{mesh.n_elements}")
    assert fe.max() <= 2e-6 and ee.max() <= 1e-5
    assert np.abs(e4 - e9).max() <= 1e-6 * np.abs(e9).max()
    # isotropic stress in the water: exact in the 4-quantity groups
    w4 = d4[wet]
    exact = np.all(w4[:, :, 1] == w4[:, :, 0], axis=1) & np.all(w4[:, :, 2] == w4[:, :, 0], axis=1) \
        & np.all(w4[:, :, 3:6] == 0.0, axis=(1, 2))
    say(f"  water elements with exactly isotropic stress: {int(exact.sum())}/{int(wet.sum())}")
    assert exact.sum() >= 16 * inf4["n_acoustic_groups"]
    scale = np.abs(w4[:, :, 0]).max()
    assert np.abs(w4[:, :, 1] - w4[:, :, 0]).max() <= 1e-5 * scale
    assert np.abs(w4[:, :, 3:6]).max() <= 1e-5 * scale
