"""Autotuned launch configurations of the matrix-core kernels.

The tuner times predictor and corrector launch configurations (wavefronts per
work-group, persistent-grid size, XCD-contiguous order, the corrector's
passes over its output rows) and the predictor's shape (FP32: I~ parked in
LDS or in HBM; BF16: 16x16x16 or gfx950's 16x16x32 products over two row
tiles) at set-up and keeps the fastest in a cache file.
Every configuration performs the same products in the same order per output,
but the compiled instruction streams differ, so results agree to rounding:
per-field relative L2 below 2e-6 (FP32, a tenth of the FP32 parity bar) or
1e-3 (BF16, where a changed last bit can flip an operand's BF16 rounding).
"""
import numpy as np
import pytest

from paper_2107_06640_amd import inputs

pytestmark = pytest.mark.gpu


def box():
    return inputs.coupled_box(6, 6, 4, cell=500.0, water_layers=1, jitter=0.1, seed=7)


def run(mesh, mats, precision, steps=2):
    from paper_2107_06640_amd import seis
    s = seis.from_mesh(mesh, mats, 6, precision=precision, kernel="tuned", mc_min=0)
    try:
        q = inputs.random_dofs(mesh.n_elements, s.B, seed=3, acoustic=mats[2] == 0)
        s.write(q)
        s.run(steps)
        return s.read()[0], s.info()
    finally:
        s.close()


def test_autotune_measures_then_reads_cache(tmp_path, monkeypatch):
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("SEIS_TUNE_CACHE", str(cache))
    monkeypatch.delenv("SEIS_TUNE", raising=False)
    mesh, mats = box()
    _, i1 = run(mesh, mats, "fp32", steps=0)
    assert i1["launch_source"] == 1
    w, cap, rm = i1["launch"][:3]
    assert w in (2, 4) and 0 <= cap <= 8 and rm in (0, 1) and i1["launch"][6] in (1, 2)
    lines = cache.read_text().splitlines()
    assert len(lines) == 1 and "/N5/p1/" in lines[0] and len(lines[0].split()) == 9
    assert i1["shape"] in (0, 1) and int(lines[0].split()[8]) == i1["shape"]
    _, i2 = run(mesh, mats, "fp32", steps=0)
    assert i2["launch_source"] == 2 and i2["launch"] == i1["launch"] and i2["shape"] == i1["shape"]
    _, i3 = run(mesh, mats, "bf16", steps=0)   # another key: measured again
    assert i3["launch_source"] == 1
    assert len(cache.read_text().splitlines()) == 2


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_launch_configurations_agree(tmp_path, monkeypatch, precision):
    mesh, mats = box()
    monkeypatch.setenv("SEIS_TUNE_CACHE", str(tmp_path / "tune.txt"))
    outs = []
    for cfg in ("4,0,0,4,0,0,2", "2,1,1,2,2,1,1", "4,2,1,2,4,0,2", "2,0,0,4,1,1,1", "4,1,1,4,1,1,1,1",
                "2,0,1,4,0,0,2,1", None):
        if cfg is None:
            monkeypatch.delenv("SEIS_TUNE", raising=False)
        else:
            monkeypatch.setenv("SEIS_TUNE", cfg)
        d, inf = run(mesh, mats, precision)
        if cfg is not None:
            c = [int(x) for x in cfg.split(",")]
            assert inf["launch"][:7] == c[:7] and inf["launch_source"] == 0
            assert inf["shape"] == (c[7] if len(c) > 7 else 0)
        outs.append(d)
    tol = 2e-6 if precision == "fp32" else 1e-3
    ref = outs[0]
    nrm = np.sqrt((ref ** 2).sum(axis=(0, 1)))
    for d in outs[1:]:
        rel = np.sqrt(((d - ref) ** 2).sum(axis=(0, 1))) / nrm
        print(precision, "max field difference", rel.max())
        assert rel.max() < tol


@pytest.mark.parametrize("shape", [0, 1])
@pytest.mark.parametrize("precision,tol", [("fp32", 2e-5), ("bf16", 3e-2)])
def test_every_predictor_shape_matches_the_oracle(monkeypatch, precision, tol, shape):
    """Each shape the tuner chooses among, fixed through SEIS_TUNE, against the
    FP64 oracle on the graded LTS box (orders 6 and 7: 16x16x32 products over
    pairs of row tiles and a lone last tile)."""
    from paper_2107_06640_amd import seis
    from tests.parity_util import field_errors, oracle_for
    zn = np.array([0.0, 0.5, 0.75, 0.875, 0.9375, 0.96875, 1.0]) * 1000.0 - 1000.0
    mesh, mats = inputs.coupled_box(4, 4, 6, cell=500.0, water_layers=1, z_nodes=zn, jitter=0.1, seed=2)
    monkeypatch.setenv("SEIS_TUNE", f"4,1,1,4,1,1,1,{shape}")
    for order in (6, 7):
        o = oracle_for(mesh, mats, order, max_clusters=4)
        q = inputs.random_dofs(mesh.n_elements, o.B, seed=order, acoustic=mats[2] == 0)
        o.Q[:] = q
        o.run(2)
        s = seis.from_mesh(mesh, mats, order, precision=precision, kernel="tuned", max_clusters=4, mc_min=0)
        try:
            assert s.info()["shape"] == shape
            s.write(q)
            s.run(2)
            d, _ = s.read()
        finally:
            s.close()
        fe = field_errors(d, o.Q)
        print(f"case: {precision} shape {shape} order {order}: max field error {fe.max():.2e}", flush=True)
        assert fe.max() < tol
