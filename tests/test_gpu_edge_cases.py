"""Edge cases of the element update, through the C ABI, against the oracle.

* An empty mesh and a mesh with a zero-volume element are rejected at set-up
  with SEIS_EINVAL and a message naming the problem.
* A single tetrahedron with four absorbing faces (every face a boundary, no
  neighbour) and a single one with four rigid-wall faces: FP64 plain at
  1e-10 and FP32 on the matrix-core kernels (one 16-element group with 15
  padding lanes, mc_min = 0) at the FP32 bars of the other parity tests.
* Ragged element counts around the 16-element group size (17 and 31
  elements, cut from a jittered box with every boundary kind): FP32
  matrix-core kernels against the oracle per field and per element.
* The zero state is a fixed point: Q = 0 and eta = 0 stay exactly zero for
  every precision and kernel (the update is linear and has no source).
"""
import sys

import numpy as np
import pytest

from paper_2107_06640_amd import inputs
from tests.parity_util import element_errors, field_errors, oracle_for

pytestmark = pytest.mark.gpu

TOL = {"fp64": (1e-10, 1e-9), "fp32": (6e-6, 2.5e-5)}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def one_tet(kind):
    xyz = np.array([[0.0, 0.0, 0.0], [900.0, 100.0, 0.0], [150.0, 1000.0, 50.0], [100.0, 200.0, 800.0]])
    tet = np.array([[0, 1, 2, 3]], dtype=np.int64)
    fk = np.full((1, 4), kind, dtype=np.int8)
    return inputs.Mesh(xyz, tet, fk, np.zeros(3))


def sub_box(n_keep):
    """The first n_keep tetrahedra of a jittered box; faces whose neighbour is cut become absorbing."""
    m = inputs.box_mesh(3, 2, 2, lengths=(3000.0, 2000.0, 2000.0), jitter=0.2, seed=7,
                        sides={"x-": "absorbing", "x+": "wall", "y-": "free", "y+": "free",
                               "z-": "absorbing", "z+": "wall"})
    from oracle.mesh import adjacency
    nb, _, _ = adjacency(m.tet, m.face_kind, m.xyz, m.period)
    fk = m.face_kind[:n_keep].copy()
    cut = nb[:n_keep] >= n_keep  # neighbour element cut away
    fk[cut] = inputs.FACE_ABSORBING
    return inputs.Mesh(m.xyz, m.tet[:n_keep].copy(), fk, np.zeros(3))


def run_pair(mesh, mats, order, steps, precision, kernel, seed):
    from paper_2107_06640_amd import seis
    o = oracle_for(mesh, mats, order)
    q = inputs.random_dofs(mesh.n_elements, o.B, seed=seed)
    o.Q[:] = q
    o.run(steps)
    s = seis.from_mesh(mesh, mats, order, precision=precision, kernel=kernel, mc_min=0)
    try:
        s.write(q)
        s.run(steps)
        d, _ = s.read()
    finally:
        s.close()
    return field_errors(d, o.Q, o.geo.absdet), element_errors(d, o.Q)


def test_empty_and_degenerate_meshes_rejected():
    from paper_2107_06640_amd import seis
    mats = (np.zeros(0), np.zeros(0), np.zeros(0))
    empty = inputs.Mesh(np.zeros((0, 3)), np.zeros((0, 4), np.int64), np.zeros((0, 4), np.int8), np.zeros(3))
    with pytest.raises(seis.SeisError) as ex:
        seis.from_mesh(empty, mats, 4)
    assert ex.value.code == -1 and "empty" in str(ex.value)
    flat = one_tet(inputs.FACE_ABSORBING)
    flat.xyz[3] = 0.3 * flat.xyz[1] + 0.3 * flat.xyz[2]  # fourth vertex in the plane of the others
    m1 = inputs.uniform_materials(flat, 2700.0, 6000.0, 3464.0)
    with pytest.raises(seis.SeisError) as ex:
        seis.from_mesh(flat, m1, 4)
    assert ex.value.code == -1 and "degenerate" in str(ex.value)


@pytest.mark.parametrize("kind", [inputs.FACE_ABSORBING, inputs.FACE_WALL])
@pytest.mark.parametrize("precision,kernel", [("fp64", "plain"), ("fp32", "tuned")])
def test_single_element(kind, precision, kernel):
    mesh = one_tet(kind)
    mats = inputs.uniform_materials(mesh, 2700.0, 6000.0, 3464.0)
    say(f"case: one tet, face kind {kind}, order 5, {precision}/{kernel}, 5 steps")
    fe, ee = run_pair(mesh, mats, 5, 5, precision, kernel, seed=3)
    say(f"  field {fe.max():.2e} element {ee.max():.2e}")
    assert fe.max() <= TOL[precision][0] and ee.max() <= TOL[precision][1]


@pytest.mark.parametrize("n_keep", [17, 31])
def test_ragged_groups(n_keep):
    mesh = sub_box(n_keep)
    mats = inputs.uniform_materials(mesh, 2500.0, 5000.0, 2800.0)
    say(f"case: {n_keep} tets of a jittered box, order 6, fp32/tuned, 4 steps")
    fe, ee = run_pair(mesh, mats, 6, 4, "fp32", "tuned", seed=n_keep)
    say(f"  field {fe.max():.2e} element {ee.max():.2e}")
    assert fe.max() <= TOL["fp32"][0] and ee.max() <= TOL["fp32"][1]


@pytest.mark.parametrize("precision,kernel", [("fp64", "plain"), ("fp32", "tuned"), ("bf16", "tuned"),
                                              ("bf16x3", "tuned")])
def test_zero_state_is_a_fixed_point(precision, kernel):
    from paper_2107_06640_amd import seis
    zn = np.array([0.0, 0.6, 0.85, 0.95, 1.0]) * 1000.0 - 1000.0
    mesh, mats = inputs.coupled_box(2, 2, 4, cell=500.0, water_layers=1, z_nodes=zn)
    say(f"case: zero state, coupled LTS box, order 5, {precision}/{kernel}")
    s = seis.from_mesh(mesh, mats, 5, precision=precision, kernel=kernel, max_clusters=3, mc_min=0)
    try:
        inf = s.info()
        s.write(np.zeros((mesh.n_elements, inf["n_basis"], 9)), np.zeros((inf["n_gravity_faces"], inf["n_eta_points"])))
        s.run(3)
        d, e = s.read()
    finally:
        s.close()
    assert not d.any() and not e.any()
