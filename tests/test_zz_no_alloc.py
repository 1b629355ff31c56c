"""seis_energy_noalloc (partial sums in the library's fixed device array)
against seis_energy (partial sums in a buffer the library allocates).

Both launch the same kernels on the same grid, so the results must agree
bit for bit. Two calls in a row on two handles, the second on a smaller
mesh (fewer work-groups, so the fixed array keeps stale partial sums of the
first call beyond what the second reads), each checked against seis_energy
of its own handle; then the first handle again after the second.
"""
import sys

import numpy as np
import pytest

from paper_2107_06640_amd import inputs

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def energy(s, noalloc):
    import torch
    out = torch.full((12,), float("nan"), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    s.energy_into(out.data_ptr(), noalloc=noalloc)
    s.sync()
    return out.cpu().numpy()


@pytest.mark.parametrize("precision,kernel", [("fp64", "plain"), ("fp32", "tuned")])
def test_noalloc_energy_matches_allocating_entry_point(precision, kernel):
    from paper_2107_06640_amd import seis
    big_mesh, big_mats = inputs.coupled_box(12, 10, 8, cell=500.0, water_layers=2, jitter=0.1, seed=1)
    small_mesh, small_mats = inputs.coupled_box(3, 2, 2, cell=500.0, water_layers=1, jitter=0.1, seed=2)
    handles = []
    try:
        for mesh, mats, seed in ((big_mesh, big_mats, 5), (small_mesh, small_mats, 6)):
            s = seis.from_mesh(mesh, mats, 4, precision=precision, kernel=kernel, mc_min=0)
            handles.append(s)
            s.write(inputs.random_dofs(mesh.n_elements, s.B, seed=seed, acoustic=mats[2] == 0),
                    np.random.default_rng(seed).standard_normal((s.n_gravity_faces, s.nq)))
            s.step()
        big, small = handles
        say(f"case: no-alloc energy {precision}/{kernel}: E={big.E} then E={small.E}")
        results = []
        for s in (big, small, big):
            a = energy(s, noalloc=True)
            b = energy(s, noalloc=False)
            say(f"  E={s.E}: noalloc {a[0]:.17e} alloc {b[0]:.17e}")
            assert np.all(np.isfinite(a))
            assert np.array_equal(a, b)
            results.append(a)
        assert np.array_equal(results[0], results[2])
        assert results[1][0] < results[0][0]
    finally:
        for s in handles:
            s.close()
