"""Option validation of seis_setup on the host.

seis_setup checks its options before it looks for a device, so malformed
options are rejected with SEIS_EINVAL (-1) and a message naming the option
even where no GPU is present.
"""
import os

import pytest

from paper_2107_06640_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2107_06640_amd", "libseis.so")


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
@pytest.mark.parametrize("kw,order,word", [
    (dict(mc_min=-1), 4, "mc_min"),
    (dict(precision="bf16", kernel="plain"), 4, "BF16"),
    (dict(), 9, "order"),
    (dict(), 1, "order"),
    (dict(precision="fp32"), 2, "3..7"),
    (dict(precision="bf16"), 8, "3..7"),
    (dict(precision="bf16x3"), 7, "3..6"),
])
def test_setup_rejects_bad_options(kw, order, word):
    from paper_2107_06640_amd import seis
    mesh, mats = inputs.coupled_box(2, 2, 2, cell=500.0, water_layers=1)
    with pytest.raises(seis.SeisError) as ex:
        seis.from_mesh(mesh, mats, order, **kw)
    assert ex.value.code == -1
    assert word in str(ex.value)


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_default_options():
    import ctypes as C
    from paper_2107_06640_amd import seis
    lib = seis.load_library()
    opt = seis.Options_t()
    lib.seis_default_options(C.byref(opt))
    assert opt.precision == 0 and opt.kernel == 0 and opt.max_clusters == 1
    assert abs(opt.cfl - 0.35) < 1e-15 and abs(opt.g - 9.81) < 1e-15
    assert opt.tile == 0 and opt.graph == 0 and opt.mc_min == 2048
    assert opt.fused == 1 and opt.acoustic == 1
