"""Parity on the 192k-element coupled box with a gravity surface, full size.

Workload: 40 x 40 x 20 cubes x 6 tets (192 000 elements), 500 m cells, top
quarter water over elastic rock, gravity free surface on top, absorbing
bottom, periodic sides; order 5 (B = 35), global time stepping; FP64 on the
plain kernels and FP32 on the matrix-core kernels. The oracle cannot run the
whole mesh, so after one time step sampled elements are compared with the
oracle run on their patch (element + face neighbours) for the same step:
their update depends only on the patch (Sec. 4.1 and 4.2: one element's
update reads its own predictor and its face neighbours' traces). Samples
cover gravity faces, the elastic-acoustic seafloor, absorbing and periodic
faces and plain interior elements; eta of the sampled gravity faces is
compared too.

Tolerance: relative L2 of each sampled element's DOFs (and of eta): FP64
1e-10 (the bar of the small parity cases), FP32 1e-4 (as at the 2M-element
size).
"""
import numpy as np
import pytest

from oracle.mesh import Geometry, adjacency
from oracle.solver import Oracle
from paper_2107_06640_amd import inputs
from tests.parity_util import submesh

pytestmark = pytest.mark.gpu

ORDER = 5
N = ORDER - 1
CFL = 0.35
CASES = [("fp64", "plain", 1e-10), ("fp32", "tuned", 1e-4)]


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def box():
    mesh, mats = inputs.cfg2()
    rho, lam, mu = mats
    geo = Geometry(mesh.xyz, mesh.tet)
    nb, _, _ = adjacency(mesh.tet, mesh.face_kind, mesh.xyz, mesh.period)
    cp = np.sqrt((lam + 2 * mu) / rho)
    dt = float((CFL / (2 * N + 1) * geo.h / cp).min())

    fk = mesh.face_kind
    wet = mu == 0
    seafloor = np.zeros(mesh.n_elements, bool)
    for f in range(4):
        j = np.maximum(nb[:, f], 0)
        seafloor |= (nb[:, f] >= 0) & (wet != wet[j])
    rng = np.random.default_rng(5)
    groups = {
        "gravity": np.any(fk == inputs.FACE_GRAVITY, axis=1),
        "seafloor": seafloor,
        "absorbing": np.any(fk == inputs.FACE_ABSORBING, axis=1),
        "periodic": np.any(fk == inputs.FACE_PERIODIC, axis=1),
        "interior": np.all(fk == inputs.FACE_INTERIOR, axis=1) & ~seafloor,
    }
    ids = np.unique(np.concatenate([rng.choice(np.nonzero(m)[0], 12, replace=False) for m in groups.values()]))

    B = (N + 1) * (N + 2) * (N + 3) // 6
    blk = inputs.random_dofs(4096, B, seed=2)
    q = np.tile(blk, (-(-mesh.n_elements // 4096), 1, 1))[: mesh.n_elements]
    q[wet, :, 1] = q[wet, :, 0]
    q[wet, :, 2] = q[wet, :, 0]
    q[wet, :, 3:6] = 0.0

    sub, smats, ring, pos = submesh(mesh, mats, ids)
    o = Oracle(sub.xyz, sub.tet, sub.face_kind, sub.period, *smats, N, cfl=CFL,
               cluster_of=np.zeros(ring.size, np.int64), dt_min=dt)
    o.Q[:] = q[ring]
    o.run(1)
    ge, gf = np.nonzero(fk == inputs.FACE_GRAVITY)
    g_index = {(int(e), int(f)): k for k, (e, f) in enumerate(zip(ge, gf))}
    sample = set(ids.tolist())
    eta_pairs = [(g_index[(int(ring[e]), int(f))], k)
                 for k, (e, f) in enumerate(zip(o.grav_elem, o.grav_face)) if int(ring[e]) in sample]
    say(f"coupled box E={mesh.n_elements} dt={dt:.4e} samples={ids.size} patch={ring.size} "
        f"gravity samples={len(eta_pairs)}")
    return dict(mesh=mesh, mats=mats, dt=dt, ids=ids, q=q, ref_q=o.Q[pos], eta_pairs=eta_pairs, ref_eta=o.eta)


@pytest.mark.parametrize("precision,kernel,tol", CASES)
def test_coupled_box_sampled_against_oracle(box, precision, kernel, tol):
    from paper_2107_06640_amd import seis
    say(f"case: coupled box 192k order {ORDER} {precision}/{kernel}")
    s = seis.from_mesh(box["mesh"], box["mats"], ORDER, precision=precision, kernel=kernel, cfl=CFL)
    try:
        inf = s.info()
        assert inf["n_clusters"] == 1
        assert abs(inf["dt_min"] - box["dt"]) <= 1e-13 * box["dt"]
        s.write(box["q"])
        s.step()
        got = s.read_elements(box["ids"])
        _, eta = s.read(dofs=False)
    finally:
        s.close()
    ref = box["ref_q"]
    err = np.sqrt(((got - ref) ** 2).sum(axis=(1, 2)) / (ref ** 2).sum(axis=(1, 2)))
    say(f"{precision}: per-element relative L2 max {err.max():.2e} median {np.median(err):.2e}")
    assert err.max() < tol
    gi = [a for a, _ in box["eta_pairs"]]
    oi = [b for _, b in box["eta_pairs"]]
    ref_eta = box["ref_eta"][oi]
    ee = np.linalg.norm(eta[gi] - ref_eta) / np.linalg.norm(ref_eta)
    say(f"{precision}: eta relative L2 {ee:.2e}")
    assert ee < tol


# 200 steps from seeded seafloor pulses: reduced precision against FP64
STEPS = 200
BAR = {"fp32": 1e-4, "bf16x3": 3e-3, "bf16": 1.0}


def test_200_steps_reduced_precision_against_fp64():
    """The 192k-element box as its workload is stated: a seeded sum of three
    Gaussian v_z pulses (widths 2-5 cells) at the seafloor, 200 global time
    steps. The FP64 path (plain kernels, pinned to the oracle by the sampled
    test above) is the reference; FP32, split BF16 and BF16 operands on the
    matrix-core kernels are compared per field (relative L2 with |det J|
    weights, each field against its own norm) and on eta. Bars: FP32 1e-4
    (its round-off accumulates to about 1e-5 here), split BF16 3e-3 (17-bit
    operands), BF16 reported with the sanity bar 1 (8-bit operands; its
    accuracy is compared with the discretisation error in the accuracy tests)."""
    from paper_2107_06640_amd import seis
    mesh, mats = inputs.cfg2()
    X = mesh.xyz[mesh.tet]
    w = np.abs(np.linalg.det(np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]], axis=2)))
    B = (ORDER) * (ORDER + 1) * (ORDER + 2) // 6
    q = inputs.pulse_dofs(mesh, B, mesh.info["z_seafloor"], 500.0, seed=0)

    def run(precision, kernel):
        say(f"case: 192k box order {ORDER} {precision}/{kernel} {STEPS} steps")
        s = seis.from_mesh(mesh, mats, ORDER, precision=precision, kernel=kernel, cfl=CFL)
        try:
            s.write(q)
            s.run(STEPS)
            return s.read()
        finally:
            s.close()

    ref, ref_eta = run("fp64", "plain")
    nrm = np.sqrt(np.einsum("e,ebp->p", w, ref ** 2))
    assert np.all(nrm > 0) and np.abs(ref_eta).max() > 0
    for prec in ("fp32", "bf16x3", "bf16"):
        d, eta = run(prec, "tuned")
        rel = np.sqrt(np.einsum("e,ebp->p", w, (d - ref) ** 2)) / nrm
        ee = np.linalg.norm(eta - ref_eta) / np.linalg.norm(ref_eta)
        say(f"  {prec}: per field " + " ".join(f"{x:.1e}" for x in rel) + f"; eta {ee:.1e}")
        assert rel.max() <= BAR[prec] and ee <= BAR[prec]
