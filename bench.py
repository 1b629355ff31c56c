"""Throughput of the ADER-DG element update on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision fp32|fp64|bf16|bf16x3]
                    [--kernel tuned|plain] [--order 6] [--scale 1] [--no-cpu-baseline]

Workload: the graded, jittered ocean-over-solid box (72 x 72 x 64 cubes x 6 =
1 990 656 tetrahedra; 500 m horizontal cells, vertical layers graded from
500 m to 125 m toward the sea surface, top quarter water with a gravity
surface), order 6 (B = 56), rate-2 LTS with up to 4 clusters. A step is one
LTS macro step; the element updates of a macro step are sum_c n_c 2^(C-1-c).
Inputs (mesh data, DOFs) are resident in HBM before the timed region.

Prints one JSON line with the metric, a roofline object for the dominant
kernel (event-timed on the library's stream) and the CPU oracle timed on a
bounded sample of the same workload. An FP32 run adds the same measurement
with BF16 operands ("bf16") and with split BF16 operands ("bf16x3").
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {  # MI355X published peaks
    "hbm_GBs": 8000.0,
    "fp64_TF": 78.6,
    "fp32_TF": 157.3,
    "bf16_TF": 2500.0,
}
BYTES = {"fp64": 8, "fp32": 4, "bf16": 4, "bf16x3": 4}


def nb(N):
    return (N + 1) * (N + 2) * (N + 3) // 6


def nf(N):
    return (N + 1) * (N + 2) // 2


def algorithmic_counts(N, value_bytes, acoustic=False):
    """Per-element algorithmic flops and HBM bytes of the predictor and corrector kernels.

    Nine-quantity form. Flops: CK with shrinking support (star matrices at 24
    non-zeros), the time integral, the volume term over the B_{N-1} non-zero
    columns of K^d, face traces and lifts at B_f nodes (2 B_f B 9 each per
    face) and the pointwise Riemann solve (9 x 9 per node). Bytes: what the
    executed form must move at least once: the predictor reads Q, G (9),
    material (3) and the own-trace flux coefficients (4 x 12) and writes Q and
    the 4 B_f x 9 traces it hands over; the corrector reads its 4 B_f x 9
    inbox, material, the neighbour-trace coefficients (4 x 12) and reads and
    writes Q.

    4-quantity form (acoustic=True, s_xx = -p and the velocity): 4 columns in
    every contraction, star matrices at 18 non-zeros (per direction three in
    the pressure row, one in each velocity row), the own-trace Riemann solve
    4 x 4 and the neighbour-trace one 4 x 9 per node; Q and the traces at 4
    values per row.
    """
    B, Bf, B1 = nb(N), nf(N), nb(N - 1)
    q = 4 if acoustic else 9
    nz = 18 if acoustic else 72
    ck = sum(2 * 3 * nb(N - k - 1) * nb(N - k) * q + 2 * nb(N - k - 1) * nz for k in range(N))
    tint = sum(2 * nb(N - k) * q for k in range(N + 1))
    traces = 2 * 4 * Bf * B * q
    flux_own = 2 * 4 * Bf * q * q
    flux_nb = 2 * 4 * Bf * q * 9
    volume = 2 * B1 * nz + 2 * B * 3 * B1 * q
    lift = 2 * 4 * B * Bf * q
    pred_flops = ck + tint + traces + flux_own + volume + lift
    corr_flops = flux_nb + lift
    vb = value_bytes
    pred_bytes = vb * (B * q + 12 + 4 * 12 + 4 * Bf * q + B * q)
    corr_bytes = vb * (4 * Bf * q + 3 + 4 * 12 + 2 * B * q)
    return dict(pred_flops=pred_flops, corr_flops=corr_flops, pred_bytes=pred_bytes, corr_bytes=corr_bytes)


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_cfg3_order6.json")


def kernel_source_hash():
    """Hash of the library sources (the one the autotuner keys its cache on)."""
    from paper_2107_06640_amd.build import source_hash
    return source_hash()


def measured_traffic(kernel_kind, precision, kernel, order):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3 counters.

    The counters (FETCH_SIZE and WRITE_SIZE, scaled by the copy calibration)
    were taken on the benchmark workload; they are used only while the
    kernel sources still hash to the value recorded with them, else None.
    """
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("source_hash") != kernel_source_hash() or kernel != "tuned" or order != rec.get("order"):
        return None
    v = rec.get("per_launch_bytes", {}).get(precision, {}).get(kernel_kind)
    return None if v is None else float(v)


WORKLOADS = {
    # the benchmark box: +-20% jitter leaves one outlier element as the
    # finest cluster, so nearly every element steps with the coarsest step
    "cfg3": 0.2,
    # the same box with +-10% jitter: three clusters that each carry a real
    # share of the updates (LTS saves a third of them)
    "cfg3-lts": 0.1,
    # rock box of 64 x 64 x 32 cubes (786 432 tets, 500 m cells, +-10%
    # jitter) with a dynamic-rupture fault at mid-depth: 8192 fault faces
    # under a background traction above the static strength (the whole
    # fault slips), and the same mesh welded (fault faces interior)
    "fault": 0.1,
    "fault-welded": 0.1,
}

# friction of the fault workload: s0 = -50 MPa, tau0 = 31 MPa along x,
# mu_s 0.6, mu_d 0.5, D_c 0.4 m, no cohesion
FAULT_PARAMS = [-50e6, 31e6, 0.0, 0.0, 0.6, 0.5, 0.4, 0.0]


def workload(scale, seed=0, name="cfg3"):
    from paper_2107_06640_amd import inputs
    if name.startswith("fault"):
        n = 64 // scale
        mesh, mats = inputs.fault_box(n, n, n // 2, cell=500.0, k_fault=n // 4, jitter=WORKLOADS[name], seed=seed)
        if name == "fault-welded":
            mesh.face_kind[mesh.face_kind == inputs.FACE_FAULT] = inputs.FACE_INTERIOR
        return mesh, mats
    mesh, mats = inputs.cfg3(scale=scale, seed=seed, jitter=WORKLOADS[name])
    return mesh, mats


def tiled_dofs(E, B, seed, wet):
    """Random DOFs for E elements by tiling a seeded block (throughput input)."""
    from paper_2107_06640_amd import inputs
    blk = min(E, 8192)
    base = inputs.random_dofs(blk, B, seed=seed)
    reps = -(-E // blk)
    q = np.tile(base, (reps, 1, 1))[:E]
    q[wet, :, 1] = q[wet, :, 0]
    q[wet, :, 2] = q[wet, :, 0]
    q[wet, :, 3:6] = 0.0
    return q


def precision_sweep(args):
    """Per-field error of FP32, split BF16 and BF16 against FP64, and throughput, at orders 4-7.

    The benchmark mesh, 504 sub-steps of dt_min (63 macro steps of 8), from
    seeded Gaussian v_z pulses at the seafloor. The FP64 reference is the
    library's FP64 path (plain kernels), the one the parity tests pin to the
    oracle. Prints one JSON line per (order, precision).
    """
    import torch
    from paper_2107_06640_amd import inputs, seis
    mesh, mats = workload(args.scale)
    X = mesh.xyz[mesh.tet]
    J = np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]], axis=2)
    w = np.abs(np.linalg.det(J))
    del X, J
    z_floor = mesh.info["z_seafloor"]
    macro = args.sweep_steps
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()

    def run(order, precision, kernel, q):
        s = seis.from_mesh(mesh, mats, order, precision=precision, kernel=kernel, max_clusters=args.max_clusters,
                           stream=stream.cuda_stream)
        inf = s.info()
        s.write(q)
        s.sync()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        s.run(macro)
        b.record(stream)
        b.synchronize()
        d, e = s.read()
        s.close()
        sub = macro * (1 << (inf["n_clusters"] - 1))
        return d, e, inf["updates_per_macro_step"] * macro / (a.elapsed_time(b) / 1e3), sub

    for order in args.sweep_orders:
        B = (order) * (order + 1) * (order + 2) // 6
        q = inputs.pulse_dofs(mesh, B, z_floor, 500.0, seed=0)
        ref, ref_eta, ups, sub = run(order, "fp64", "plain", q)
        nrm = np.sqrt(np.einsum("e,ebp->p", w, ref ** 2))
        print(json.dumps({"order": order, "precision": "fp64", "kernel": "plain", "substeps": sub,
                          "updates_per_s": ups}), flush=True)
        for prec in ("fp32", "bf16x3", "bf16") if order <= 6 else ("fp32", "bf16"):
            d, eta, ups, _ = run(order, prec, "tuned", q)
            err = np.sqrt(np.einsum("e,ebp->p", w, (d - ref) ** 2))
            rel = err / np.where(nrm > 0, nrm, nrm.max())
            ee = float(np.linalg.norm(eta - ref_eta) / max(np.linalg.norm(ref_eta), 1e-300))
            print(json.dumps({"order": order, "precision": prec, "kernel": "tuned", "substeps": sub,
                              "updates_per_s": ups, "rel_l2_per_field": [float(x) for x in rel],
                              "rel_l2_eta": ee}), flush=True)
            del d
        del ref


def host_description():
    """nproc, CPU model and memory of the host (for the CPU baseline record)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    mem_gb = None
    try:
        with open("/proc/meminfo") as f:
            for line in f:
                if line.startswith("MemTotal"):
                    mem_gb = round(int(line.split()[1]) / 2 ** 20, 1)
                    break
    except OSError:
        pass
    return {"nproc": len(os.sched_getaffinity(0)), "cpu_model": model, "mem_GiB": mem_gb}


def cpu_baseline(order, budget_s=15.0):
    """Oracle element-updates/s on a 6 x 6 x 8-cube sample of the workload (GTS)."""
    from oracle.solver import Oracle
    from paper_2107_06640_amd import inputs
    zn = inputs.graded_z_nodes(8, 500.0, 250.0)
    mesh, mats = inputs.coupled_box(6, 6, 8, cell=500.0, water_layers=2, z_nodes=zn, jitter=0.2, seed=0)
    rho, lam, mu = mats
    o = Oracle(mesh.xyz, mesh.tet, mesh.face_kind, mesh.period, rho, lam, mu, order - 1)
    o.Q[:] = inputs.random_dofs(mesh.n_elements, o.B, seed=0, acoustic=mu == 0)
    o.run(1)  # warm caches
    t0 = time.perf_counter()
    u0 = o.updates
    n = 0
    while time.perf_counter() - t0 < budget_s:
        o.run(1)
        n += 1
    dt = time.perf_counter() - t0
    try:
        from threadpoolctl import threadpool_info
        cores = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count() or 1
    return dict(value=(o.updates - u0) / dt, unit="element-updates/s", cores=int(cores), kind="oracle",
                host=host_description(),
                sample=f"{mesh.n_elements} tets (6x6x8 cubes of the graded coupled box, order {order}, "
                       f"global time stepping), {n} steps in {dt:.1f} s")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="fp32", choices=["fp64", "fp32", "bf16", "bf16x3"])
    ap.add_argument("--kernel", default="tuned", choices=["tuned", "plain"])
    ap.add_argument("--order", type=int, default=6)
    ap.add_argument("--scale", type=int, default=1)
    ap.add_argument("--workload", default="cfg3", choices=sorted(WORKLOADS))
    ap.add_argument("--per-cluster", action="store_true",
                    help="one launch per cluster instead of one per phase per sub-step")
    ap.add_argument("--max-clusters", type=int, default=4)
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--mc-min", type=int, default=None,
                    help="clusters with fewer elements run on the plain FP32 kernels (library default 2048)")
    ap.add_argument("--graph", action="store_true",
                    help="replay each macro step as one hipGraph; kernel timings then come from a "
                         "separate eagerly launched pass of the same length")
    ap.add_argument("--nine-quantity-water", action="store_true",
                    help="acoustic elements in the nine-quantity embedding everywhere (no 4-quantity groups)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-bf16", action="store_true",
                    help="FP32 runs: skip the BF16 and split-BF16 measurements reported beside the FP32 line")
    ap.add_argument("--sweep", action="store_true",
                    help="precision sweep: FP32/split BF16/BF16 against FP64 at orders 4-7 (one JSON line each)")
    ap.add_argument("--sweep-orders", type=int, nargs="+", default=[4, 5, 6, 7])
    ap.add_argument("--sweep-steps", type=int, default=63, help="macro steps (63 x 8 = 504 sub-steps)")
    ap.add_argument("--copy-probe", type=float, default=0.0,
                    help="only run a device-to-device copy of this many GiB (counter calibration)")
    args = ap.parse_args()

    if args.copy_probe > 0:
        import torch
        n = int(args.copy_probe * (1 << 30)) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": 4 * n, "copy_probe_bytes_written": 4 * n, "copies": 3}),
              flush=True)
        return

    if args.sweep:
        precision_sweep(args)
        return

    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the method would shard by domain decomposition, see the design notes)", file=sys.stderr)
        sys.exit(2)

    import torch

    mesh, mats = workload(args.scale, name=args.workload)
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    run = measure(args, mesh, mats, args.precision, stream)
    inf, ms, eager_ms, prof = run["info"], run["ms"], run["eager_ms"], run["prof"]
    value = inf["updates_per_macro_step"] * args.steps / (ms / 1e3)
    roof = roofline(args, args.precision, inf, prof)

    out = {
        "metric": "ADER-DG element-updates/s (order 6), FP32/BF16 vs FP64, % of roofline",
        "value": value,
        "unit": "element-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[args.precision],
        "data": "synthetic",
        "config": {"workload": workload_description(args, inf),
                   "kernel": args.kernel, "precision": args.precision, "elements": inf["n_elements"],
                   "graph": bool(args.graph), "fused": bool(inf["fused"]),
                   "eager_ms_per_step": eager_ms / args.steps,
                   "launches_per_step": {k: v[1] / args.steps for k, v in prof.items()},
                   "launch": launch_record(args.precision, inf),
                   "acoustic_groups": inf["n_acoustic_groups"],
                   "acoustic_fraction": acoustic_fraction(inf),
                   "updates_per_step": inf["updates_per_macro_step"]},
        "roofline": roof,
        "kernels_ms": {k: v[0] for k, v in prof.items()},
    }
    if args.precision == "fp32" and args.kernel == "tuned" and not args.no_bf16:
        # the BF16-operand kernels (and, up to order 6, split BF16 operands)
        # on the same workload, same steps and timing
        for prec in ("bf16", "bf16x3") if args.order <= 6 else ("bf16",):
            b = measure(args, mesh, mats, prec, stream)
            bi = b["info"]
            out[prec] = {
                "value": bi["updates_per_macro_step"] * args.steps / (b["ms"] / 1e3),
                "ms_per_step": b["ms"] / args.steps,
                "dtype": DTYPE[prec],
                "launch": launch_record(prec, bi),
                "roofline": roofline(args, prec, bi, b["prof"]),
                "kernels_ms": {k: v[0] for k, v in b["prof"].items()},
            }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.order)
    print(json.dumps(out), flush=True)


DTYPE = {"fp64": "f64", "fp32": "f32", "bf16": "bf16-in/f32-acc", "bf16x3": "split-bf16-in (hi+lo, 3 products)/f32-acc"}


def workload_description(args, inf):
    if args.workload.startswith("fault"):
        what = (f"rock box with a mid-depth dynamic-rupture fault, {inf['n_fault_faces']} fault faces slipping"
                if args.workload == "fault" else "rock box, the fault plane welded (interior faces)")
    else:
        what = "graded jittered ocean-over-solid box"
    return (f"{args.workload}: {what} (jitter {WORKLOADS[args.workload]}), {inf['n_elements']} tets, "
            f"order {args.order} (B={inf['n_basis']}), rate-2 LTS {inf['n_clusters']} clusters "
            f"{inf['cluster_size']}, {inf['n_gravity_faces']} gravity faces")


def measure(args, mesh, mats, precision, stream):
    """Set up the solver, warm up, and time args.steps macro steps on the library's stream.

    Returns the solver info, the event-timed milliseconds of the timed steps
    (graph replays with --graph), those of an eagerly launched pass, and the
    per-kernel profile (milliseconds, launches, elements) of the eager pass.
    """
    import torch
    from paper_2107_06640_amd import seis

    t_setup = time.perf_counter()
    s = seis.from_mesh(mesh, mats, args.order, precision=precision, kernel=args.kernel,
                       max_clusters=args.max_clusters, stream=stream.cuda_stream, tile=args.tile,
                       graph=args.graph, mc_min=args.mc_min, fused=not args.per_cluster,
                       acoustic=not args.nine_quantity_water)
    try:
        inf = s.info()
        if inf["n_fault_faces"]:
            s.set_fault(FAULT_PARAMS)
        q = tiled_dofs(mesh.n_elements, inf["n_basis"], 0, mats[2] == 0)
        s.write(q)
        del q
        t_setup = time.perf_counter() - t_setup
        print(f"# {precision}: setup {t_setup:.1f} s, E={inf['n_elements']}, clusters={inf['cluster_size']}, "
              f"updates/macro={inf['updates_per_macro_step']}, 4-quantity groups={inf['n_acoustic_groups']}",
              file=sys.stderr, flush=True)

        for _ in range(args.warmup):
            s.step()
        s.sync()
        torch.cuda.synchronize()

        def timed_steps(profile):
            s.profile(profile)
            start = torch.cuda.Event(enable_timing=True)
            stop = torch.cuda.Event(enable_timing=True)
            start.record(stream)
            for _ in range(args.steps):
                s.step()
            stop.record(stream)
            stop.synchronize()
            torch.cuda.synchronize()
            prof = s.profile_read() if profile else None
            s.profile(False)
            return start.elapsed_time(stop), prof

        if args.graph:
            ms, _ = timed_steps(False)       # graph replays
            eager_ms, prof = timed_steps(True)
        else:
            ms, prof = timed_steps(True)
            eager_ms = ms
        return dict(info=inf, ms=ms, eager_ms=eager_ms, prof=prof)
    finally:
        s.close()


def acoustic_fraction(inf):
    """Share of the elements that sit in 16-element groups of the 4-quantity form."""
    return min(1.0, 16.0 * inf["n_acoustic_groups"] / inf["n_elements"])


def launch_record(precision, inf):
    return {"predict": inf["launch"][:3], "correct": inf["launch"][3:7], "mc_min": inf["launch"][7],
            "predict_shape": {("fp32", 0): "I~ park LDS", ("fp32", 1): "I~ park HBM",
                              ("bf16", 0): "bf16 16x16x16", ("bf16", 1): "bf16 16x16x32",
                              ("bf16x3", 0): "split bf16 16x16x16"}.get(
                                  (precision, inf["shape"]), "plain"),
            "source": ["default", "measured", "cache"][inf["launch_source"]]}


def roofline(args, precision, inf, prof):
    """Roofline object of the dominant kernel from its event-timed launches.

    The algorithmic work per element is that of the form the element runs
    in: the acoustic_fraction of the elements count with the 4-quantity
    figures, the rest with the nine-quantity ones.
    """
    N = args.order - 1
    c9 = algorithmic_counts(N, BYTES[precision])
    c4 = algorithmic_counts(N, BYTES[precision], acoustic=True)
    fa = acoustic_fraction(inf) if args.kernel == "tuned" and precision != "fp64" else 0.0
    cnt = {k: (1.0 - fa) * c9[k] + fa * c4[k] for k in c9}
    pms, pl, pe = prof["predict"]
    cms, cl, ce = prof["correct"]
    dom = "predict" if pms >= cms else "correct"
    kms, kl, ke = prof[dom]
    flops = cnt["pred_flops" if dom == "predict" else "corr_flops"] * ke / kl
    byts = cnt["pred_bytes" if dom == "predict" else "corr_bytes"] * ke / kl
    avg_s = kms / kl / 1e3
    peak_tf = PEAK[{"fp64": "fp64_TF", "fp32": "fp32_TF", "bf16": "bf16_TF", "bf16x3": "bf16_TF"}[precision]]
    t_flop = flops / (peak_tf * 1e12)
    t_byte = byts / (PEAK["hbm_GBs"] * 1e9)
    if t_flop >= t_byte:
        bound = "mfma" if args.kernel == "tuned" else "alu"
        roof = dict(bound=bound, achieved=flops / avg_s / 1e12, peak=peak_tf, unit="TFLOP/s")
    else:
        roof = dict(bound="hbm", achieved=byts / avg_s / 1e9, peak=PEAK["hbm_GBs"], unit="GB/s")
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = measured_traffic(dom, precision, args.kernel, args.order) \
        if args.workload == "cfg3" else None
    roof["traffic_source"] = ("stored rocprofv3 FETCH_SIZE/WRITE_SIZE of these kernel sources "
                              "(profiles/traffic_cfg3_order6.json)") if roof["traffic"] is not None else None
    roof["kernel"] = dom
    roof["avg_launch_ms"] = kms / kl
    roof["flops_per_launch"] = flops
    roof["bytes_per_launch"] = byts
    return roof


if __name__ == "__main__":
    main()
