"""Parity at the full benchmark size, in the benchmark's launch configuration.

Workload: the graded, jittered ocean-over-solid box of 72 x 72 x 64 cubes
(1 990 656 tetrahedra), order 6, rate-2 LTS with at most 4 clusters, tuned
kernels, as timed by bench.py. The oracle cannot run the whole mesh, so:

* the LTS cluster of every element (Sec. 4.4 reading: floor(log2(dt/dt_min))
  capped, neighbours at most one cluster apart) is compared bit-exactly with
  the oracle's assignment on the full mesh;
* after one macro step, sampled elements of the coarsest cluster whose face
  neighbours are all in that cluster are compared with the oracle run on the
  patch (element + face neighbours) for one step of 8 dt_min, the coarsest
  cluster's step: their update depends only on the patch. Samples cover
  gravity faces, the elastic-acoustic seafloor, absorbing and periodic faces
  and plain interior elements. eta of the sampled gravity faces is compared
  too.

Tolerance: relative L2 of each sampled element's DOFs (and eta) against the
oracle. FP32 operands: 1e-4 (an element's own round-off is about 1e-6 of
its norm; cancellation in the update of small elements costs up to two
orders more). Split BF16 operands: 5e-4 (an operand keeps 2^-18 of its
value, about 4e-6, with the same two orders for cancellation). BF16
operands: 3e-2, as for the small parity cases.
"""
import numpy as np
import pytest

from oracle.mesh import Geometry, adjacency
from oracle.solver import Oracle, assign_clusters
from paper_2107_06640_amd import inputs
from tests.parity_util import submesh

pytestmark = pytest.mark.gpu

ORDER = 6
N = ORDER - 1
C_MAX = 4
CFL = 0.35
TOL = {"fp32": 1e-4, "bf16x3": 5e-4, "bf16": 3e-2}


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def full():
    mesh, mats = inputs.cfg3()
    rho, lam, mu = mats
    geo = Geometry(mesh.xyz, mesh.tet)
    nb, _, _ = adjacency(mesh.tet, mesh.face_kind, mesh.xyz, mesh.period)
    cp = np.sqrt((lam + 2 * mu) / rho)
    dt_elem = CFL / (2 * N + 1) * geo.h / cp
    cl, dt_min = assign_clusters(dt_elem, nb, C_MAX)
    top = cl.max()

    # samples: coarsest-cluster elements whose face neighbours share the cluster
    ok = cl == top
    for f in range(4):
        ok &= (nb[:, f] < 0) | (cl[np.maximum(nb[:, f], 0)] == top)
    fk = mesh.face_kind
    wet = mu == 0
    seafloor = np.zeros(mesh.n_elements, bool)
    for f in range(4):
        j = np.maximum(nb[:, f], 0)
        seafloor |= (nb[:, f] >= 0) & (wet != wet[j])
    rng = np.random.default_rng(11)
    groups = {
        "gravity": ok & np.any(fk == inputs.FACE_GRAVITY, axis=1),
        "seafloor": ok & seafloor,
        "absorbing": ok & np.any(fk == inputs.FACE_ABSORBING, axis=1),
        "periodic": ok & np.any(fk == inputs.FACE_PERIODIC, axis=1),
        "interior": ok & np.all(fk == inputs.FACE_INTERIOR, axis=1) & ~seafloor,
    }
    ids = np.unique(np.concatenate([rng.choice(np.nonzero(m)[0], 12, replace=False) for m in groups.values()]))

    # seeded DOFs: one random block tiled over the mesh (as the benchmark does)
    blk = inputs.random_dofs(8192, (N + 1) * (N + 2) * (N + 3) // 6, seed=0)
    q = np.tile(blk, (-(-mesh.n_elements // 8192), 1, 1))[: mesh.n_elements]
    q[wet, :, 1] = q[wet, :, 0]
    q[wet, :, 2] = q[wet, :, 0]
    q[wet, :, 3:6] = 0.0

    # oracle on the patch around the samples, one step of the coarsest cluster
    sub, smats, ring, pos = submesh(mesh, mats, ids)
    o = Oracle(sub.xyz, sub.tet, sub.face_kind, sub.period, *smats, N, cfl=CFL,
               cluster_of=np.zeros(ring.size, np.int64), dt_min=dt_min * 2 ** top)
    o.Q[:] = q[ring]
    o.run(1)
    ref_q = o.Q[pos]
    # eta of the samples' gravity faces: global order is (element, local face)
    ge, gf = np.nonzero(fk == inputs.FACE_GRAVITY)
    g_index = {(int(e), int(f)): k for k, (e, f) in enumerate(zip(ge, gf))}
    eta_pairs = [(g_index[(int(ring[e]), int(f))], k)
                 for k, (e, f) in enumerate(zip(o.grav_elem, o.grav_face)) if int(ring[e]) in set(ids.tolist())]
    say(f"full mesh E={mesh.n_elements} clusters={np.bincount(cl).tolist()} samples={ids.size} "
        f"patch={ring.size} gravity samples={len(eta_pairs)}")
    return dict(mesh=mesh, mats=mats, cl=cl, dt_min=dt_min, ids=ids, q=q, ref_q=ref_q,
                eta_pairs=eta_pairs, ref_eta=o.eta)


@pytest.mark.parametrize("precision", ["fp32", "bf16x3", "bf16"])
def test_full_size_sampled_against_oracle(full, precision):
    from paper_2107_06640_amd import seis
    s = seis.from_mesh(full["mesh"], full["mats"], ORDER, precision=precision, kernel="tuned",
                       max_clusters=C_MAX, cfl=CFL)
    try:
        assert np.array_equal(s.cluster_of(), full["cl"])
        inf = s.info()
        assert abs(inf["dt_min"] - full["dt_min"]) <= 1e-13 * full["dt_min"]
        s.write(full["q"])
        s.step()
        got = s.read_elements(full["ids"])
        _, eta = s.read(dofs=False)
    finally:
        s.close()
    ref = full["ref_q"]
    err = np.sqrt(((got - ref) ** 2).sum(axis=(1, 2)) / (ref ** 2).sum(axis=(1, 2)))
    say(f"{precision}: per-element relative L2 max {err.max():.2e} median {np.median(err):.2e}")
    assert err.max() < TOL[precision]
    gi = [a for a, _ in full["eta_pairs"]]
    oi = [b for _, b in full["eta_pairs"]]
    ref_eta = full["ref_eta"][oi]
    ee = np.linalg.norm(eta[gi] - ref_eta) / np.linalg.norm(ref_eta)
    say(f"{precision}: eta relative L2 {ee:.2e}")
    assert ee < TOL[precision]
