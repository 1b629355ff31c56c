"""Energy and field norms on the GPU (seis_energy) against the oracle.

The kernel's FP64 sums are compared with the oracle's quadrature of the same
state (the library's own state, read back): energy and per-field squared L2
norms within 1e-12 relative. The discrete energy including rho g eta^2 / 2
must not grow from one macro step to the next (upwind Godunov flux, Sec. 4.2;
gravity surface, Sec. 4.3): in FP64 within 1e-12 relative, in FP32 within
1e-6 (its state round-off).
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


def energy(s):
    import torch
    out = torch.zeros(12, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    s.energy_into(out.data_ptr())
    s.sync()
    return out.cpu().numpy()


@pytest.mark.parametrize("precision,kernel", [("fp64", "plain"), ("fp32", "tuned")])
def test_energy_matches_oracle_quadrature(precision, kernel):
    from paper_2107_06640_amd import seis
    mesh, mats = lts_box()
    o = oracle_for(mesh, mats, 5, max_clusters=4)
    s = seis.from_mesh(mesh, mats, 5, precision=precision, kernel=kernel, max_clusters=4, mc_min=0)
    try:
        say(f"case: energy {precision}/{kernel} order 5")
        q = inputs.random_dofs(mesh.n_elements, o.B, seed=1, acoustic=mats[2] == 0)
        eta = np.random.default_rng(2).standard_normal(o.eta.shape) * 0.1
        s.write(q, eta)
        s.run(2)
        d, e = s.read()
        got = energy(s)
    finally:
        s.close()
    E = o.energy(Q=d, eta=e)
    Es = o.energy(Q=np.zeros_like(d), eta=e)
    nrm = o.field_sq_norms(d)
    say(f"  E {got[0]:.6e} oracle {E:.6e}; surface {got[2]:.6e} oracle {Es:.6e}")
    assert abs(got[0] - E) <= 1e-12 * E
    assert abs(got[2] - Es) <= 1e-12 * Es
    assert abs(got[1] - (E - Es)) <= 1e-12 * E
    np.testing.assert_allclose(got[3:], nrm, rtol=1e-12)


@pytest.mark.parametrize("precision,kernel,tol", [("fp64", "plain", 1e-12), ("fp32", "tuned", 1e-6)])
def test_energy_never_grows(precision, kernel, tol):
    from paper_2107_06640_amd import seis
    mesh, mats = lts_box()
    s = seis.from_mesh(mesh, mats, 6, precision=precision, kernel=kernel, max_clusters=4, mc_min=0)
    try:
        say(f"case: energy decay {precision}/{kernel} order 6")
        q = inputs.random_dofs(mesh.n_elements, s.B, seed=3, acoustic=mats[2] == 0)
        eta = np.random.default_rng(4).standard_normal((s.n_gravity_faces, s.nq)) * 0.1
        s.write(q, eta)
        E = [energy(s)[0]]
        for _ in range(8):
            s.step()
            E.append(energy(s)[0])
    finally:
        s.close()
    E = np.array(E)
    say("  relative changes", np.array2string(np.diff(E) / E[0], precision=2))
    assert np.all(np.diff(E) <= tol * E[0])
    assert E[-1] < E[0]


def test_energy_rejects_mid_step():
    from paper_2107_06640_amd import seis
    mesh, mats = lts_box()
    s = seis.from_mesh(mesh, mats, 4, precision="fp32", kernel="tuned", max_clusters=4)
    try:
        s.predict(0)
        with pytest.raises(seis.SeisError) as ex:
            energy(s)
        assert ex.value.code == -4
    finally:
        s.close()
