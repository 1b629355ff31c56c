"""Reduced-precision error against the discretisation error, on the GPU.

The acceptance reading for FP32 and BF16 operands: their difference from the
library's FP64 path (which the parity tests pin to the oracle at 1e-10)
should not exceed the FP64 discretisation error, i.e. the FP64 result's
distance from the exact solution at the same resolution. Two closed-form
cases (exact solutions from oracle.analytic):

* an elastic P + S plane wave on the periodic unit cube of 6 x 6 x 6 cubes x
  6 tetrahedra (k = 2 pi (1, 0, 1)), orders 3-7, 100 time steps;
* the acoustic-gravity standing wave of a 1 km water layer over a rigid
  bottom (8 x 1 x 2 cubes of 500 m, g raised to 400 m/s^2 so that a quarter
  gravity period is a few hundred steps), orders 3-7, 300 time steps,
  DOFs and the sea-surface height eta.

Errors are physical L2 norms per field (oracle quadrature of the state read
back from the library), divided by the exact solution's norm of all stress
(or all velocity) fields together, taken at t = 0 and, for the standing wave,
also a quarter period later (its velocity vanishes at t = 0 and its pressure
a quarter period later).
Every row is printed; the accuracy table of the design notes is this output.

Findings the assertions encode:
* FP32 stays within the larger of the FP64 discretisation error and its own
  round-off floor of 2e-6 (about 30 units of FP32 round-off): at orders 6-7
  the standing wave's FP64 error (1e-7 to 1e-8) is below what FP32 can hold.
* BF16 operands (8 significant bits) leave errors of about 1e-2, above the
  FP64 discretisation error from order 4 on; the bound below (5e-2) only
  guards against regressions.
* Split BF16 operands (hi + lo, three BF16 products per product, orders 3-6)
  keep about 17 significant bits per operand (|x - hi - lo| <= 2^-18 |x|):
  within the larger of the FP64 discretisation error and a 5e-5 floor.
"""
import math
import sys

import numpy as np
import pytest

from oracle import analytic
from paper_2107_06640_amd import inputs
from tests.parity_util import oracle_for

pytestmark = pytest.mark.gpu

ROCK = inputs.lame(2700.0, 6000.0, 3464.0)
FIELDS = ["sxx", "syy", "szz", "sxy", "syz", "sxz", "vx", "vy", "vz"]
FP32_FLOOR = 2e-6
SPLIT_FLOOR = 5e-5
BF16_BOUND = 5e-2


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def l2_fields(o, Q, fn, t):
    """Per-field L2 norm of (Q - exact) and of exact, by the oracle's volume quadrature."""
    x = o.geo.x0[:, None, :] + np.einsum("edc,qc->eqd", o.geo.J, o.vpts)
    ex = fn(x.reshape(-1, 3), t).reshape(o.E, -1, 9)
    num = np.einsum("qb,ebp->eqp", o.phi_v, Q)
    w = o.geo.absdet[:, None] * o.vw[None, :]
    err = np.sqrt(np.sum(w[..., None] * (num - ex) ** 2, axis=(0, 1)))
    ref = np.sqrt(np.sum(w[..., None] * ex ** 2, axis=(0, 1)))
    return err, ref


def group_norm(ref):
    """Normalisation per field: the norm of its group (stresses 0-5, velocities 6-8)."""
    s = np.linalg.norm(ref[:6])
    v = np.linalg.norm(ref[6:])
    return np.array([s] * 6 + [v] * 3)


def run(mesh, mats, order, steps, q0, eta0, precision, kernel, cfl, g):
    from paper_2107_06640_amd import seis
    s = seis.from_mesh(mesh, mats, order, precision=precision, kernel=kernel, cfl=cfl, g=g, mc_min=0)
    try:
        s.write(q0, eta0)
        s.run(steps)
        d, e = s.read()
        return d, e, s.info()["time"]
    finally:
        s.close()


CASES = []


def study(name, mesh, mats, order, steps, fn, cfl, g=9.81, eta_fn=None, norm_times=(0.0,)):
    o = oracle_for(mesh, mats, order, cfl=cfl, g=g)
    q0 = o.project(lambda x: fn(x, 0.0))
    eta0 = None
    pts = None
    if eta_fn is not None:
        pts = o.eta_points()
        eta0 = eta_fn(pts.reshape(-1, 3), 0.0).reshape(pts.shape[:2])
    out = {}
    precs = [("fp64", "plain"), ("fp32", "tuned"), ("bf16", "tuned")] + ([("bf16x3", "tuned")] if order <= 6 else [])
    for prec, kern in precs:
        out[prec] = run(mesh, mats, order, steps, q0, eta0, prec, kern, cfl, g)
    t = out["fp64"][2]
    err64, _ = l2_fields(o, out["fp64"][0], fn, t)
    nrm = np.max([group_norm(l2_fields(o, np.zeros_like(q0), fn, tn)[1]) for tn in norm_times], axis=0)
    disc = err64 / nrm
    row = {"case": name, "order": order, "steps": steps, "t": t, "fp64_vs_exact": disc}
    reduced = [p for p, _ in precs if p != "fp64"]
    for prec in reduced:
        diff, _ = l2_fields(o, out[prec][0] - out["fp64"][0], lambda x, tt: np.zeros((x.shape[0], 9)), t)
        row[prec + "_vs_fp64"] = diff / nrm
    if eta_fn is not None:
        ex = eta_fn(pts.reshape(-1, 3), t).reshape(pts.shape[:2])
        sc = np.abs(eta0).max()
        row["eta"] = {"fp64_vs_exact": np.abs(out["fp64"][1] - ex).max() / sc}
        for prec in reduced:
            row["eta"][prec + "_vs_fp64"] = np.abs(out[prec][1] - out["fp64"][1]).max() / sc
    CASES.append(row)
    fmt = lambda v: " ".join(f"{x:.1e}" for x in v)
    say(f"| {name} | {order} | fp64-exact {fmt(disc)} |")
    for prec in reduced:
        say(f"|   | | {prec}-fp64 {fmt(row[prec + '_vs_fp64'])} |")
    if eta_fn is not None:
        say(f"|   | | eta: fp64-exact {row['eta']['fp64_vs_exact']:.1e} "
            + " ".join(f"{p}-fp64 {row['eta'][p + '_vs_fp64']:.1e}" for p in reduced) + " |")
    return row


@pytest.mark.parametrize("order", [3, 4, 5, 6, 7])
def test_plane_wave_precision_within_discretisation_error(order):
    mesh = inputs.cfg1_mesh(6)
    mats = inputs.uniform_materials(mesh, 2700.0, 6000.0, 3464.0)
    lam, mu, rho = ROCK[1], ROCK[2], ROCK[0]
    fn = analytic.plane_wave(lam, mu, rho, m=(1, 0, 1), a_p=1.0, a_s=1.0)
    say(f"case: plane wave order {order}")
    row = study("plane wave 6^3", mesh, mats, order, 100, fn, cfl=0.5)
    # the stress fields of the wave all carry energy; v_y of this wave is zero
    live = [0, 1, 2, 3, 5, 6, 8]
    assert np.all(row["fp64_vs_exact"][live] < 0.1)
    assert np.all(row["fp32_vs_fp64"][live] <= np.maximum(row["fp64_vs_exact"][live], FP32_FLOOR))
    assert np.all(row["bf16_vs_fp64"][live] <= BF16_BOUND)
    if "bf16x3_vs_fp64" in row:
        assert np.all(row["bf16x3_vs_fp64"][live] <= np.maximum(row["fp64_vs_exact"][live], SPLIT_FLOOR))


@pytest.mark.parametrize("order", [3, 4, 5, 6, 7])
def test_standing_wave_precision_within_discretisation_error(order):
    H, Lx, g = 1000.0, 4000.0, 400.0
    sw = analytic.StandingWave(1000.0, 1500.0, g, H, Lx, P=1.0e4)
    mesh = inputs.box_mesh(8, 1, 2, lengths=(Lx, 500.0, 0.0), z_nodes=-500.0 * (2 - np.arange(3)),
                           sides={"z-": "wall", "z+": "gravity"})
    mats = inputs.uniform_materials(mesh, 1000.0, 1500.0, 0.0)
    say(f"case: standing wave order {order}")
    row = study("standing wave", mesh, mats, order, 300, sw.q, cfl=0.35, g=g, eta_fn=sw.eta,
                norm_times=(0.0, 0.5 * math.pi / sw.w))
    live = [0, 1, 2, 6, 8]
    assert np.all(row["fp64_vs_exact"][live] < 0.1)
    assert np.all(row["fp32_vs_fp64"][live] <= np.maximum(row["fp64_vs_exact"][live], FP32_FLOOR))
    assert row["eta"]["fp32_vs_fp64"] <= max(row["eta"]["fp64_vs_exact"], FP32_FLOOR)
    assert np.all(row["bf16_vs_fp64"][live] <= BF16_BOUND) and row["eta"]["bf16_vs_fp64"] <= BF16_BOUND
    if "bf16x3_vs_fp64" in row:
        assert np.all(row["bf16x3_vs_fp64"][live] <= np.maximum(row["fp64_vs_exact"][live], SPLIT_FLOOR))
        assert row["eta"]["bf16x3_vs_fp64"] <= max(row["eta"]["fp64_vs_exact"], SPLIT_FLOOR)
