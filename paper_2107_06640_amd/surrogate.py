"""Learned surrogate of the coupled solver: seafloor uplift -> sea-surface height.

    python -m paper_2107_06640_amd.surrogate [--runs 64] [--steps 400] [--out DIR]

1. Data: solver runs (seis.h, FP32 matrix-core kernels) on the ocean-over-solid
   box of 24 x 24 x 12 cubes of 1 km (41 472 tets, top quarter water, gravity
   surface), order 4, each started from a seeded uplift (1-4 Gaussians,
   amplitude 0.5-3 m, width 2-6 km, rise time 5-30 s) imposed as the initial
   vertical velocity (mean uplift rate) of the rock under the seafloor. eta is
   read at the gravity-face points at 32 output times and interpolated onto a
   64 x 64 grid.
2. Network (fno.FNO): input channels = uplift rate on the 64 x 64 grid
   (repeated over the 32 times) and the three normalised coordinates x, y, t;
   output eta on the 64 x 64 x 32 grid. Trained with Adam on the relative L2
   loss, BF16 products, FP32 master weights.
3. Evaluation: relative L2 of the surrogate against the solver on held-out
   runs, and time per sample of each.
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np


def face_points(mesh, order):
    """Physical (x, y) of the eta points of every gravity face, library order.

    The points are the collapsed Gauss rule the library documents for eta:
    s = (1 + a_i)(1 - b_j)/4, t = (1 + b_j)/2 on the face parametrised by its
    vertices in ascending local order (a Gauss-Legendre, b Gauss-Jacobi(1,0),
    N + 1 points each, index j (N + 1) + i).
    """
    from scipy.special import roots_jacobi, roots_legendre
    n = order  # N + 1 points
    a, _ = roots_legendre(n)
    b, _ = roots_jacobi(n, 1.0, 0.0)
    S = np.array([(1 + a[i]) * (1 - b[j]) / 4 for j in range(n) for i in range(n)])
    T = np.array([(1 + b[j]) / 2 for j in range(n) for i in range(n)])
    ge, gf = np.nonzero(mesh.face_kind == 2)
    fv = np.array([[1, 2, 3], [0, 2, 3], [0, 1, 3], [0, 1, 2]])[gf]
    X = mesh.xyz[mesh.tet[ge[:, None], fv]]                      # [F, 3 vertices, 3]
    P = X[:, None, 0] + S[None, :, None] * (X[:, None, 1] - X[:, None, 0]) + T[None, :, None] * (X[:, None, 2] - X[:, None, 0])
    return P[..., :2].reshape(-1, 2)


class GridSampler:
    """Linear interpolation of scattered eta values onto a regular grid (nearest value outside the hull)."""

    def __init__(self, pts, gx, gy):
        from scipy.spatial import Delaunay
        self.tri = Delaunay(pts)
        q = np.stack(np.meshgrid(gx, gy, indexing="ij"), -1).reshape(-1, 2)
        s = self.tri.find_simplex(q)
        inside = s >= 0
        Tm = self.tri.transform[s[inside]]
        bary = np.einsum("nij,nj->ni", Tm[:, :2], q[inside] - Tm[:, 2])
        self.w = np.concatenate([bary, 1 - bary.sum(1, keepdims=True)], 1)
        self.idx = self.tri.simplices[s[inside]]
        self.inside = inside
        from scipy.spatial import cKDTree
        self.near = cKDTree(pts).query(q[~inside])[1]
        self.shape = (gx.size, gy.size)

    def __call__(self, vals):
        out = np.empty(self.inside.size)
        out[self.inside] = (vals[self.idx] * self.w).sum(1)
        out[~self.inside] = vals[self.near]
        return out.reshape(self.shape)


def generate(n_runs, *, grid=64, nt=32, t_end=64.0, order=4, scale=1, seed0=0, log=print):
    """Solver runs -> (uplift rate on the grid [n][G][G], eta [n][G][G][nt], seconds per run)."""
    import torch
    from . import inputs, seis
    mesh, mats = inputs.cfg5(scale=scale)
    lx, ly = mesh.xyz[:, 0].max(), mesh.xyz[:, 1].max()
    gx = (np.arange(grid) + 0.5) * lx / grid
    gy = (np.arange(grid) + 0.5) * ly / grid
    sampler = GridSampler(face_points(mesh, order), gx, gy)
    elastic = mats[2] > 0
    z_floor = mesh.info["z_seafloor"]
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    s = seis.from_mesh(mesh, mats, order, precision="fp32", kernel="tuned", max_clusters=4,
                       stream=stream.cuda_stream, graph=True)
    inf = s.info()
    dt_macro = inf["dt_min"] * (1 << (inf["n_clusters"] - 1))
    t_out = (np.arange(nt) + 1) * t_end / nt
    steps_at = np.maximum(1, np.round(t_out / dt_macro).astype(int))
    U = np.zeros((n_runs, grid, grid), np.float32)
    H = np.zeros((n_runs, grid, grid, nt), np.float32)
    secs = []
    GX, GY = np.meshgrid(gx, gy, indexing="ij")
    for r in range(n_runs):
        src = inputs.uplift_sources(seed0 + r, lx, ly)
        U[r] = inputs.uplift_rate(GX, GY, src)
        q = inputs.uplift_dofs(mesh, inf["n_basis"], z_floor, src, 1000.0 / scale, elastic)
        s.write(q, np.zeros((inf["n_gravity_faces"], inf["n_eta_points"])))
        s.sync()
        t0 = time.perf_counter()
        done = 0
        for k, n in enumerate(steps_at):
            s.run(int(n - done))
            done = n
            _, eta = s.read(dofs=False)
            H[r, :, :, k] = sampler(eta.reshape(-1))
        secs.append(time.perf_counter() - t0)
        if r % 8 == 0 or r == n_runs - 1:
            log(f"run {r}: {len(src)} sources, {secs[-1]:.2f} s, max |eta| {np.abs(H[r]).max():.3f} m")
    s.close()
    return U, H, float(np.mean(secs)), dict(mesh_elements=int(mesh.n_elements), order=order, t_end=t_end,
                                               dt_macro=dt_macro, macro_steps=int(steps_at[-1]),
                                               updates_per_macro_step=int(inf["updates_per_macro_step"]))


def make_input(U, nt):
    """[n][G][G] uplift rate -> [4][n][G][G][nt]: rate (scaled), x, y, t in [0, 1]."""
    n, G, _ = U.shape
    out = np.empty((4, n, G, G, nt), np.float32)
    out[0] = U[..., None] / max(float(np.abs(U).max()), 1e-30)
    c = (np.arange(G) + 0.5) / G
    tt = (np.arange(nt) + 1) / nt
    out[1] = c[None, :, None, None]
    out[2] = c[None, None, :, None]
    out[3] = tt[None, None, None, :]
    return out


def train(U, H, *, n_train, n_val, width=32, modes=12, layers=4, hidden=128, steps=400, batch=64, lr=1e-3,
          seed=0, log=print):
    """Train an FNO on the first n_train runs; returns (net, history, output scale)."""
    import torch
    from .fno import FNO
    n, G, _, nt = H.shape
    net = FNO(G, G, nt, cin=4, width=width, modes=modes, layers=layers, hidden=hidden, seed=seed)
    scale = float(np.abs(H[:n_train]).max())
    X = torch.tensor(make_input(U, nt), device="cuda:0")
    Y = torch.tensor(H[None] / scale, device="cuda:0")
    rng = np.random.default_rng(seed)
    hist = []
    b = min(batch, n_train)
    t0 = time.perf_counter()
    for it in range(steps):
        idx = torch.tensor(np.sort(rng.choice(n_train, b, replace=False)), device="cuda:0")
        xb = X[:, idx].contiguous()
        yb = Y[:, idx].contiguous()
        yhat = net.forward(xb, keep=True)
        loss, grad = net.loss(yhat, yb)
        net.backward(grad)
        net.adam_step(lr=lr * (0.5 * (1 + np.cos(np.pi * it / steps))))
        if it % 25 == 0 or it == steps - 1:
            val = evaluate(net, X, Y, range(n_train, n_train + n_val)) if n_val else float("nan")
            hist.append((it, float(loss[0]), val))
            log(f"step {it}: train {float(loss[0]):.4f} val {val:.4f} ({time.perf_counter() - t0:.1f} s)")
    return net, hist, scale, X, Y


def evaluate(net, X, Y, ids, batch=16):
    """Mean relative L2 of the network on runs ids."""
    import torch
    ids = list(ids)
    tot = 0.0
    for i in range(0, len(ids), batch):
        sel = torch.tensor(ids[i:i + batch], device="cuda:0")
        yhat = net.forward(X[:, sel].contiguous())
        loss, _ = net.loss(yhat, Y[:, sel].contiguous(), grad=False)
        tot += float(loss[0]) * len(sel)
    return tot / len(ids)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--runs", type=int, default=64)
    ap.add_argument("--test", type=int, default=8)
    ap.add_argument("--val", type=int, default=4)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--grid", type=int, default=64)
    ap.add_argument("--nt", type=int, default=32)
    ap.add_argument("--t-end", type=float, default=64.0)
    ap.add_argument("--width", type=int, default=32)
    ap.add_argument("--modes", type=int, default=12)
    ap.add_argument("--layers", type=int, default=4)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--out", default="surrogate_out")
    ap.add_argument("--save-data", action="store_true", help="also write the generated runs (data.npz)")
    args = ap.parse_args()
    import torch
    os.makedirs(args.out, exist_ok=True)
    log = lambda *a: print(*a, flush=True)  # noqa: E731
    U, H, solver_s, meta = generate(args.runs, grid=args.grid, nt=args.nt, t_end=args.t_end, log=log)
    if args.save_data:
        np.savez_compressed(os.path.join(args.out, "data.npz"), U=U, H=H)
    n_train = args.runs - args.test - args.val
    net, hist, scale, X, Y = train(U, H, n_train=n_train, n_val=args.val, width=args.width, modes=args.modes,
                                   layers=args.layers, steps=args.steps, batch=args.batch, log=log)
    test_ids = range(n_train + args.val, args.runs)
    err = evaluate(net, X, Y, test_ids)
    # surrogate time per sample (batched inference, after one warm-up)
    sel = torch.tensor(list(test_ids), device="cuda:0")
    xb = X[:, sel].contiguous()
    net.forward(xb)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        net.forward(xb)
    torch.cuda.synchronize()
    sur_s = (time.perf_counter() - t0) / 3 / len(sel)
    zero_err = 1.0  # predicting eta = 0 (no surrogate, no solver)
    out = dict(meta, runs=args.runs, train=n_train, val=args.val, test=args.test, grid=[args.grid, args.grid, args.nt],
               width=args.width, modes=args.modes, layers=args.layers, steps=args.steps,
               test_rel_l2=err, zero_baseline_rel_l2=zero_err, solver_s_per_run=solver_s,
               surrogate_s_per_sample=sur_s, speedup=solver_s / sur_s, history=hist,
               n_params=int(sum(p.numel() for p in net.params.values())))
    with open(os.path.join(args.out, "summary.json"), "w") as f:
        json.dump(out, f, indent=1)
    log(json.dumps({k: v for k, v in out.items() if k != "history"}))


if __name__ == "__main__":
    main()
