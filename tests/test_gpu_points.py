"""Output at points (receivers, sea surface, seafloor) against the oracle.

Receivers: seeded random points of the graded coupled box plus mesh vertices
and face centroids (shared by several elements: the lowest caller id
containing the point is used), located by the library and by the oracle
(oracle.solver.Oracle.locate, pinned on the CPU by the closed-form Kuhn
numbering); the elements must agree exactly and the sampled values of the
FP64 path after 3 LTS macro steps within 1e-10 of the oracle's run (relative
to the largest value of each field group). The built-in sets: the
sea-surface points equal the oracle's eta points and the seafloor points its
elastic-acoustic face points (to 1e-9 m), with the same values and eta.
FP32: the kernel's FP64 evaluation of the stored state equals the oracle's
evaluation of that state read back, to 1e-12.
"""
import sys

import numpy as np
import pytest

from paper_2107_06640_amd import inputs
from tests.parity_util import oracle_for

pytestmark = pytest.mark.gpu

ZN = np.array([0.0, 0.5, 0.75, 0.875, 0.9375, 0.96875, 1.0]) * 1000.0 - 1000.0


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def lts_box():
    return inputs.coupled_box(4, 4, 6, cell=500.0, water_layers=1, z_nodes=ZN, jitter=0.1, seed=2)


def receiver_points(mesh, rng):
    lo, hi = mesh.xyz.min(axis=0), mesh.xyz.max(axis=0)
    pts = [rng.uniform(lo + 1.0, hi - 1.0, size=(40, 3))]
    inner = np.nonzero(np.all((mesh.xyz > lo + 1.0) & (mesh.xyz < hi - 1.0), axis=1))[0]
    pts.append(mesh.xyz[rng.choice(inner, 6, replace=False)])                 # vertices: many elements
    e = rng.choice(mesh.n_elements, 6, replace=False)
    pts.append(mesh.xyz[mesh.tet[e][:, [1, 2, 3]]].mean(axis=1))              # face centroids: two elements
    return np.concatenate(pts)


def device_sample(s, set_id, n, eta=False):
    import torch
    out = torch.full((n, 9), float("nan"), dtype=torch.float64, device="cuda")
    ev = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda") if eta else None
    torch.cuda.synchronize()
    s.sample_into(set_id, out.data_ptr(), None if ev is None else ev.data_ptr())
    s.sync()
    return out.cpu().numpy(), (None if ev is None else ev.cpu().numpy())


def group_scale(v):
    return np.array([np.abs(v[..., :6]).max()] * 6 + [np.abs(v[..., 6:]).max()] * 3)


def test_receivers_and_surfaces_fp64_match_the_oracle():
    from paper_2107_06640_amd import seis
    mesh, mats = lts_box()
    order = 5
    o = oracle_for(mesh, mats, order, max_clusters=4)
    q = inputs.random_dofs(mesh.n_elements, o.B, seed=3, acoustic=mats[2] == 0)
    eta0 = np.random.default_rng(5).standard_normal(o.eta.shape) * 0.1
    o.Q[:] = q
    o.eta[:] = eta0
    pts = receiver_points(mesh, np.random.default_rng(7))
    s = seis.from_mesh(mesh, mats, order, precision="fp64", kernel="plain", max_clusters=4)
    try:
        rid = s.points(pts)
        x, elem = s.points_info(rid)
        ref_elem, _ = o.locate(pts)
        say(f"case: receivers fp64 order {order}: {pts.shape[0]} points")
        assert np.array_equal(x, pts) and np.array_equal(elem, ref_elem)
        s.write(q, eta0)
        o.run(3)
        s.run(3)
        got, _ = device_sample(s, rid, pts.shape[0])
        ref = o.sample(pts)
        err = (np.abs(got - ref) / group_scale(ref)).max()
        say(f"  receivers max error {err:.2e}")
        assert err <= 1e-10
        # sea surface: the eta points, values in the acoustic element, eta itself
        xs, es = s.points_info(seis.SEIS_POINTS_SEA_SURFACE)
        ps = o.eta_points().reshape(-1, 3)
        assert np.abs(xs - ps).max() <= 1e-9 and np.array_equal(es, np.repeat(o.grav_elem, o.gst.shape[0]))
        got, geta = device_sample(s, seis.SEIS_POINTS_SEA_SURFACE, xs.shape[0], eta=True)
        ref = o.face_sample(o.grav_elem, o.grav_face).reshape(-1, 9)
        err = (np.abs(got - ref) / group_scale(ref)).max()
        _, eta_read = s.read(dofs=False)
        say(f"  sea surface max error {err:.2e}, eta vs oracle {np.abs(geta - o.eta.ravel()).max():.2e}")
        assert err <= 1e-10 and np.array_equal(geta, eta_read.ravel())
        assert np.abs(geta - o.eta.ravel()).max() <= 1e-10 * np.abs(o.eta).max()
        # seafloor: elastic side of the elastic-acoustic faces
        fe, ff = o.seafloor_faces()
        xf, ef = s.points_info(seis.SEIS_POINTS_SEAFLOOR)
        pf = o.geo.face_points(fe, ff, o.gst).reshape(-1, 3)
        assert xf.shape[0] == pf.shape[0] and np.abs(xf - pf).max() <= 1e-9
        assert np.array_equal(ef, np.repeat(fe, o.gst.shape[0]))
        got, _ = device_sample(s, seis.SEIS_POINTS_SEAFLOOR, xf.shape[0])
        ref = o.face_sample(fe, ff).reshape(-1, 9)
        err = (np.abs(got - ref) / group_scale(ref)).max()
        say(f"  seafloor max error {err:.2e} over {xf.shape[0]} points")
        assert err <= 1e-10
    finally:
        s.close()


def test_fp32_sampling_of_the_stored_state():
    from paper_2107_06640_amd import seis
    mesh, mats = lts_box()
    o = oracle_for(mesh, mats, 6, max_clusters=4)
    pts = receiver_points(mesh, np.random.default_rng(8))
    s = seis.from_mesh(mesh, mats, 6, precision="fp32", kernel="tuned", max_clusters=4, mc_min=0)
    try:
        s.write(inputs.random_dofs(mesh.n_elements, s.B, seed=4, acoustic=mats[2] == 0))
        rid = s.points(pts)
        series = []
        for _ in range(3):
            s.step()
            got, _ = device_sample(s, rid, pts.shape[0])
            d, _ = s.read()
            ref = o.sample(pts, Q=d)
            series.append(got)
            err = (np.abs(got - ref) / group_scale(ref)).max()
            say(f"case: fp32 receivers, step error {err:.2e}")
            assert err <= 1e-12
        assert not np.array_equal(series[0], series[1])
    finally:
        s.close()


def test_point_outside_the_mesh_is_rejected():
    from paper_2107_06640_amd import seis
    mesh, mats = lts_box()
    s = seis.from_mesh(mesh, mats, 4, precision="fp32", kernel="tuned", max_clusters=4)
    try:
        with pytest.raises(seis.SeisError) as ex:
            s.points(np.array([[1.0e9, 0.0, -10.0]]))
        assert ex.value.code == -1
        with pytest.raises(seis.SeisError) as ex:
            s.points_info(5)
        assert ex.value.code == -5
    finally:
        s.close()
