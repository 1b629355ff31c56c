"""Learned surrogate of the coupled solver: seafloor uplift history -> sea-surface height.

    python -m paper_2107_06640_amd.surrogate [--runs 200] [--test 24] [--val 8] [--out DIR]

One-way linked tsunami models take the seafloor uplift as their input
(Sec. 2); the solver here computes the sea-surface height eta the uplift
raises through the elastic solid, the ocean and the gravity surface
(Sec. 3, Sec. 4.3). The surrogate learns that map.

1. Data: solver runs (seis.h, FP32 matrix-core kernels, rate-2 LTS, one
   hipGraph per macro step) on the ocean-over-solid box of 24 x 24 x 12 cubes
   of 1 km (41 472 tets, top quarter water, gravity surface), order 4, from
   rest. The bottom of the solid is a prescribed-velocity boundary driven by
   a seeded uplift history (seis_set_uplift): 1-4 Gaussians, amplitude
   0.5-3 m, width 2-6 km, rise time 5-30 s, u = sum A exp(-r^2/2w^2) S(t/T).
   The rise times exceed the 1.5 s the P wave needs from the bottom to the
   seafloor, so the seafloor follows the bottom. eta is read at the
   gravity-face points at 32 output times over 120 s and interpolated onto a
   64 x 64 grid. Several runs share the GPU at once, one solver handle per
   stream: one run of this size does not fill the chip.
2. Network (fno.FNO): input channels = the uplift u(x, y, t) on the
   64 x 64 x 32 grid (scaled by 3 m) and the coordinates x, y, t in [0, 1];
   output eta on the same grid. Adam on the relative L2 loss, BF16 products,
   FP32 master weights, batch 64.
3. Evaluation on held-out runs: relative L2 of eta against the solver, beside
   two measured baselines (eta = 0, and eta = u: the seafloor uplift copied to
   the sea surface, the usual initial condition of a decoupled tsunami
   model), time per sample, and a learning curve (test error against the
   number of training runs).
4. Use (Surrogate): inputs outside the training ranges, or outputs that are
   not finite or exceed the physically possible amplitude, are answered by
   the solver instead (the solver is the fallback and the reference that
   checks the network).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import time

import numpy as np

# training distribution of the uplift sources (inputs.uplift_sources)
RANGES = dict(count=(1, 4), amplitude=(0.5, 3.0), width=(2000.0, 6000.0), rise=(5.0, 30.0))
U_SCALE = 3.0  # m, input scaling of the uplift channel


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


def uplift_grid(sources, gx, gy, t):
    """u(x, y, t) on the grid [G][G][nt] (the same history the solver's bottom follows)."""
    X, Y = np.meshgrid(gx, gy, indexing="ij")
    out = np.zeros((gx.size, gy.size, t.size))
    for a, cx, cy, w, T in sources:
        s = np.clip(t / T, 0.0, 1.0)
        ramp = s - np.sin(2 * np.pi * s) / (2 * np.pi)
        out += a * np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / (2 * w * w))[..., None] * ramp[None, None, :]
    return out


class Solver:
    """Solver runs for lists of uplift sources: K handles on K streams, advanced together."""

    def __init__(self, *, grid=64, nt=32, t_end=120.0, order=4, scale=1, concurrent=4):
        import torch
        from . import inputs, seis
        self.torch = torch
        mesh, mats = inputs.cfg5(scale=scale, bottom="velocity")
        self.mesh, self.order, self.nt, self.t_end = mesh, order, nt, t_end
        self.lx, self.ly = float(mesh.xyz[:, 0].max()), float(mesh.xyz[:, 1].max())
        self.gx = (np.arange(grid) + 0.5) * self.lx / grid
        self.gy = (np.arange(grid) + 0.5) * self.ly / grid
        self.sampler = GridSampler(face_points(mesh, order), self.gx, self.gy)
        torch.cuda.set_device(0)
        self.streams = [torch.cuda.Stream() for _ in range(concurrent)]
        self.handles = [seis.from_mesh(mesh, mats, order, precision="fp32", kernel="tuned", max_clusters=4,
                                       stream=st.cuda_stream, graph=True) for st in self.streams]
        inf = self.handles[0].info()
        self.info = inf
        self.dt_macro = inf["dt_min"] * (1 << (inf["n_clusters"] - 1))
        self.t_out = (np.arange(nt) + 1) * t_end / nt
        self.steps_at = np.maximum(1, np.round(self.t_out / self.dt_macro).astype(int))
        self.zero_q = np.zeros((inf["n_elements"], inf["n_basis"], 9))
        self.zero_eta = np.zeros((inf["n_gravity_faces"], inf["n_eta_points"]))

    def close(self):
        for h in self.handles:
            h.close()
        self.handles = []

    def run(self, source_lists, log=None):
        """eta on the grid [n][G][G][nt] for each list of sources; wall seconds per run (amortised)."""
        n = len(source_lists)
        H = np.zeros((n, self.gx.size, self.gy.size, self.nt), np.float32)
        t0 = time.perf_counter()
        K = len(self.handles)
        for b in range(0, n, K):
            batch = list(range(b, min(n, b + K)))
            for j, r in enumerate(batch):
                h = self.handles[j]
                h.write(self.zero_q, self.zero_eta)
                h.set_uplift(np.asarray(source_lists[r], dtype=np.float64).reshape(-1, 5))
            done = 0
            for k, nsteps in enumerate(self.steps_at):
                for j, _ in enumerate(batch):
                    self.handles[j].run(int(nsteps - done))   # asynchronous on the handle's stream
                done = nsteps
                for j, r in enumerate(batch):
                    _, eta = self.handles[j].read(dofs=False)
                    H[r, :, :, k] = self.sampler(eta.reshape(-1))
            if log and (b // K) % 4 == 0:
                log(f"runs {b}-{batch[-1]}: {time.perf_counter() - t0:.1f} s, max |eta| {np.abs(H[batch]).max():.3f} m")
        return H, (time.perf_counter() - t0) / max(n, 1)


def make_input(sources, gx, gy, t, lx, ly, t_end):
    """[4][n][G][G][nt]: u / 3 m, x, y, t in [0, 1]."""
    n = len(sources)
    out = np.empty((4, n, gx.size, gy.size, t.size), np.float32)
    for r, src in enumerate(sources):
        out[0, r] = uplift_grid(src, gx, gy, t) / U_SCALE
    out[1] = (gx / lx)[None, :, None, None]
    out[2] = (gy / ly)[None, None, :, None]
    out[3] = (t / t_end)[None, None, None, :]
    return out


def in_range(sources, lx, ly):
    """The sources lie in the training distribution (count, amplitude, width, rise time, centre)."""
    c0, c1 = RANGES["count"]
    if not (c0 <= len(sources) <= c1):
        return False
    for a, cx, cy, w, T in sources:
        if not (RANGES["amplitude"][0] <= a <= RANGES["amplitude"][1] and RANGES["width"][0] <= w <= RANGES["width"][1]
                and RANGES["rise"][0] <= T <= RANGES["rise"][1]):
            return False
        mx, my = min(w, 0.45 * lx), min(w, 0.45 * ly)
        if not (mx <= cx <= lx - mx and my <= cy <= ly - my):
            return False
    return True


def train(X, Y, *, n_train, val_ids=(), width=32, modes=12, layers=4, hidden=128, steps=400, batch=64, lr=1e-3,
          seed=0, log=print):
    """Train an FNO on runs 0..n_train-1 of X [4][n]..., Y [1][n]... (device tensors)."""
    import torch
    from .fno import FNO
    _, n, G, G2, nt = X.shape
    net = FNO(G, G2, nt, cin=4, width=width, modes=modes, layers=layers, hidden=hidden, seed=seed)
    rng = np.random.default_rng(seed)
    hist = []
    b = min(batch, n_train)
    t0 = time.perf_counter()
    for it in range(steps):
        idx = torch.tensor(np.sort(rng.choice(n_train, b, replace=False)), device=X.device)
        yhat = net.forward(X[:, idx].contiguous(), keep=True)
        loss, grad = net.loss(yhat, Y[:, idx].contiguous())
        net.backward(grad)
        net.adam_step(lr=lr * (0.5 * (1 + np.cos(np.pi * it / steps))))
        if it % 50 == 0 or it == steps - 1:
            val = evaluate(net, X, Y, val_ids) if len(val_ids) else float("nan")
            hist.append((it, float(loss[0]), val))
            log(f"  step {it}: train {float(loss[0]):.4f} val {val:.4f} ({time.perf_counter() - t0:.1f} s)")
    return net, hist


def evaluate(net, X, Y, ids, batch=16):
    """Mean relative L2 of the network on runs ids."""
    import torch
    ids = list(ids)
    tot = 0.0
    for i in range(0, len(ids), batch):
        sel = torch.tensor(ids[i:i + batch], device=X.device)
        yhat = net.forward(X[:, sel].contiguous())
        loss, _ = net.loss(yhat, Y[:, sel].contiguous(), grad=False)
        tot += float(loss[0]) * len(sel)
    return tot / len(ids)


def rel_l2(a, b):
    """Mean over runs of |a - b| / |b| (axes after the first)."""
    a = a.reshape(a.shape[0], -1).astype(np.float64)
    b = b.reshape(b.shape[0], -1).astype(np.float64)
    return float(np.mean(np.linalg.norm(a - b, axis=1) / np.linalg.norm(b, axis=1)))


class Surrogate:
    """The trained network with the solver as fallback and reference."""

    def __init__(self, net, y_scale, solver, lx, ly):
        self.net, self.y_scale, self.solver, self.lx, self.ly = net, y_scale, solver, lx, ly

    def predict(self, source_lists):
        """eta [n][G][G][nt] and, per run, whether the solver answered instead of the network."""
        import torch
        s = self.solver
        ok = [in_range(src, self.lx, self.ly) for src in source_lists]
        out = np.zeros((len(source_lists), s.gx.size, s.gy.size, s.nt), np.float32)
        net_ids = [i for i, v in enumerate(ok) if v]
        if net_ids:
            X = torch.tensor(make_input([source_lists[i] for i in net_ids], s.gx, s.gy, s.t_out, s.lx, s.ly,
                                        s.t_end), device="cuda:0")
            y = self.net.forward(X).cpu().numpy()[0] * self.y_scale
            for k, i in enumerate(net_ids):
                amp = sum(abs(a) for a, *_ in source_lists[i])
                # a sea surface cannot rise more than the uplift beneath it
                if np.isfinite(y[k]).all() and np.abs(y[k]).max() <= 2.0 * amp:
                    out[i] = y[k]
                else:
                    ok[i] = False
        redo = [i for i, v in enumerate(ok) if not v]
        if redo:
            H, _ = s.run([source_lists[i] for i in redo])
            for k, i in enumerate(redo):
                out[i] = H[k]
        return out, np.array([not v for v in ok])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--runs", type=int, default=200)
    ap.add_argument("--test", type=int, default=24)
    ap.add_argument("--val", type=int, default=8)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--curve-steps", type=int, default=250)
    ap.add_argument("--curve", type=int, nargs="*", default=[21, 42, 84])
    ap.add_argument("--grid", type=int, default=64)
    ap.add_argument("--nt", type=int, default=32)
    ap.add_argument("--t-end", type=float, default=120.0)
    ap.add_argument("--width", type=int, default=32)
    ap.add_argument("--modes", type=int, default=12)
    ap.add_argument("--layers", type=int, default=4)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--concurrent", type=int, default=4)
    ap.add_argument("--out", default="surrogate_out")
    args = ap.parse_args()
    import torch
    from . import inputs
    os.makedirs(args.out, exist_ok=True)
    log = lambda *a: print(*a, flush=True)  # noqa: E731
    solver = Solver(grid=args.grid, nt=args.nt, t_end=args.t_end, concurrent=args.concurrent)
    src = [inputs.uplift_sources(r, solver.lx, solver.ly) for r in range(args.runs)]
    H, solver_s = solver.run(src, log=log)
    X = torch.tensor(make_input(src, solver.gx, solver.gy, solver.t_out, solver.lx, solver.ly, args.t_end),
                     device="cuda:0")
    n_train = args.runs - args.test - args.val
    y_scale = float(np.abs(H[:n_train]).max())
    Y = torch.tensor(H[None] / y_scale, device="cuda:0")
    val_ids = range(n_train, n_train + args.val)
    test_ids = list(range(n_train + args.val, args.runs))
    # measured baselines on the test runs: eta = 0, and eta = u (uplift copied to the surface)
    U = X[0].cpu().numpy() * U_SCALE
    base_zero = rel_l2(np.zeros_like(H[test_ids]), H[test_ids])
    base_copy = rel_l2(U[test_ids], H[test_ids])
    curve = []
    for nc in sorted(set(args.curve)):
        if nc >= n_train:
            continue
        log(f"learning curve: {nc} training runs")
        net_c, _ = train(X, Y, n_train=nc, width=args.width, modes=args.modes, layers=args.layers,
                         steps=args.curve_steps, batch=args.batch, log=log)
        curve.append((nc, evaluate(net_c, X, Y, test_ids)))
        del net_c
    log(f"final model: {n_train} training runs")
    net, hist = train(X, Y, n_train=n_train, val_ids=val_ids, width=args.width, modes=args.modes,
                      layers=args.layers, steps=args.steps, batch=args.batch, log=log)
    err = evaluate(net, X, Y, test_ids)
    curve.append((n_train, err))
    sel = torch.tensor(test_ids, device="cuda:0")
    xb = X[:, sel].contiguous()
    net.forward(xb)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        net.forward(xb)
    torch.cuda.synchronize()
    sur_s = (time.perf_counter() - t0) / 3 / len(test_ids)
    # power law err = a n^-b through the curve, extrapolated to 1600 training runs (of 2000)
    fit = None
    if len(curve) >= 3:
        lx_, ly_ = np.log([c[0] for c in curve]), np.log([c[1] for c in curve])
        b, a = np.polyfit(lx_, ly_, 1)
        fit = dict(exponent=float(b), at_1600=float(math.exp(a) * 1600 ** b))
    # the solver as fallback: an out-of-range input (amplitude 6 m) is answered by the solver
    sur = Surrogate(net, y_scale, solver, solver.lx, solver.ly)
    probe = [src[test_ids[0]], [(6.0, 12000.0, 12000.0, 4000.0, 10.0)]]
    _, used_solver = sur.predict(probe)
    info = solver.info
    out = dict(mesh_elements=int(solver.mesh.n_elements), order=4, t_end=args.t_end,
               dt_macro=solver.dt_macro, macro_steps=int(solver.steps_at[-1]),
               updates_per_macro_step=int(info["updates_per_macro_step"]), concurrent_runs=args.concurrent,
               runs=args.runs, train=n_train, val=args.val, test=args.test,
               grid=[args.grid, args.grid, args.nt], width=args.width, modes=args.modes, layers=args.layers,
               steps=args.steps, test_rel_l2=err, baseline_zero_rel_l2=base_zero, baseline_uplift_copy_rel_l2=base_copy,
               solver_s_per_run=solver_s, surrogate_s_per_sample=sur_s, speedup=solver_s / sur_s,
               learning_curve=curve, power_law=fit, fallback_probe_used_solver=[bool(v) for v in used_solver],
               history=hist, n_params=int(sum(p.numel() for p in net.params.values())))
    solver.close()
    with open(os.path.join(args.out, "summary.json"), "w") as f:
        json.dump(out, f, indent=1)
    log(json.dumps({k: v for k, v in out.items() if k != "history"}))


if __name__ == "__main__":
    main()
