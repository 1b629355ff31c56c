"""Host-side behaviour of bench.py that needs no GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=300, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def _jacobians(lam, mu, rho):
    """A_x, A_y, A_z of the velocity-stress system (quantity order s_xx s_yy s_zz s_xy s_yz s_xz v_x v_y v_z)."""
    import numpy as np
    A = np.zeros((3, 9, 9))
    l2m = lam + 2 * mu
    # stress rows: -(C grad v); velocity rows: -(div sigma)/rho
    for e, (n0, n1, n2) in enumerate(((l2m, lam, lam), (lam, l2m, lam), (lam, lam, l2m))):
        A[e, 0, 6 + e], A[e, 1, 6 + e], A[e, 2, 6 + e] = -n0, -n1, -n2
    A[0, 3, 7] = A[1, 3, 6] = -mu
    A[1, 4, 8] = A[2, 4, 7] = -mu
    A[0, 5, 8] = A[2, 5, 6] = -mu
    sig = [[0, 3, 5], [3, 1, 4], [5, 4, 2]]  # sigma_ij as a quantity index
    for i in range(3):
        for e in range(3):
            A[e, 6 + i, sig[i][e]] = -1.0 / rho
    return A


def test_star_nonzeros_behind_the_algorithmic_counts():
    """The star-matrix non-zeros the counts use (72 = 3 x 24 elastic, 18 = 3 x 6 in the
    4-quantity form) and the 4/9 scaling of every contraction, from the Jacobians."""
    import numpy as np
    sys.path.insert(0, ROOT)
    import bench
    G = np.random.default_rng(0).standard_normal((3, 3))
    el = np.einsum("de,eij->dij", G, _jacobians(2.0, 1.0, 1.5))
    ac = np.einsum("de,eij->dij", G, _jacobians(2.0, 0.0, 1.0))
    keep = [0, 6, 7, 8]
    # acoustic: s_yy = s_zz = s_xx folds their columns into column 0
    fold = ac[:, :, keep].copy()
    fold[:, :, 0] += ac[:, :, 1] + ac[:, :, 2]
    nz_el = int((np.abs(el) > 0).sum())
    nz_ac = int((np.abs(fold[:, keep, :]) > 0).sum())
    assert (nz_el, nz_ac) == (72, 18)
    N = 5
    c9, c4 = bench.algorithmic_counts(N, 4), bench.algorithmic_counts(N, 4, acoustic=True)
    B, B1 = bench.nb(N), bench.nb(N - 1)
    vol9 = 2 * B1 * nz_el + 2 * B * 3 * B1 * 9
    vol4 = 2 * B1 * nz_ac + 2 * B * 3 * B1 * 4
    ck9 = sum(2 * 3 * bench.nb(N - k - 1) * bench.nb(N - k) * 9 + 2 * bench.nb(N - k - 1) * nz_el for k in range(N))
    ck4 = sum(2 * 3 * bench.nb(N - k - 1) * bench.nb(N - k) * 4 + 2 * bench.nb(N - k - 1) * nz_ac for k in range(N))
    Bf = bench.nf(N)
    rest9 = sum(2 * bench.nb(N - k) * 9 for k in range(N + 1)) + 2 * 4 * Bf * B * 9 * 2 + 2 * 4 * Bf * 81
    rest4 = sum(2 * bench.nb(N - k) * 4 for k in range(N + 1)) + 2 * 4 * Bf * B * 4 * 2 + 2 * 4 * Bf * 16
    assert c9["pred_flops"] == ck9 + vol9 + rest9
    assert c4["pred_flops"] == ck4 + vol4 + rest4
    assert c4["corr_flops"] == 2 * 4 * Bf * 4 * 9 + 2 * 4 * B * Bf * 4
