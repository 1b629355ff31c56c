"""End to end: solver-generated data, surrogate training on the BF16 kernels,
the solver as fallback, and what the trained network gains.

A small instance of the pipeline (6 x 6 x 3 cubes of 1 km, order 3, eta on a
16 x 16 x 8 grid over 30 s, the bottom driven by seeded uplift histories):
* runs advanced together on two streams equal runs made one at a time, bit
  for bit;
* the trained network beats both measured baselines (eta = 0, and the
  uplift copied to the sea surface) on runs it has not seen, and answers
  faster per sample than the solver;
* an input outside the training ranges (a 6 m uplift) is answered by the
  solver: the surrogate returns exactly what the solver computes.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_surrogate_pipeline_with_solver_fallback():
    import time
    import torch
    from paper_2107_06640_amd import inputs, surrogate
    solver = surrogate.Solver(grid=16, nt=8, t_end=30.0, order=3, scale=4, concurrent=2)
    try:
        src = [inputs.uplift_sources(r, solver.lx, solver.ly) for r in range(24)]
        H, solver_s = solver.run(src, log=print)
        assert np.isfinite(H).all() and np.abs(H).max() > 0
        one = surrogate.Solver(grid=16, nt=8, t_end=30.0, order=3, scale=4, concurrent=1)
        try:
            H1, _ = one.run(src[:3])
        finally:
            one.close()
        assert np.array_equal(H1, H[:3])
        X = torch.tensor(surrogate.make_input(src, solver.gx, solver.gy, solver.t_out, solver.lx, solver.ly, 30.0),
                         device="cuda:0")
        y_scale = float(np.abs(H[:20]).max())
        Y = torch.tensor(H[None] / y_scale, device="cuda:0")
        net, _ = surrogate.train(X, Y, n_train=20, width=8, modes=3, layers=2, hidden=16, steps=300, batch=16,
                                 lr=3e-3, log=print)
        err = surrogate.evaluate(net, X, Y, range(20, 24))
        U = X[0].cpu().numpy() * surrogate.U_SCALE
        base_copy = surrogate.rel_l2(U[20:24], H[20:24])
        sel = torch.arange(20, 24, device="cuda:0")
        xb = X[:, sel].contiguous()
        net.forward(xb)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        net.forward(xb)
        torch.cuda.synchronize()
        sur_s = (time.perf_counter() - t0) / 4
        print(f"held-out relative L2 {err:.3f} (uplift copied to the surface: {base_copy:.3f}); "
              f"solver {solver_s:.3f} s/run, surrogate {sur_s * 1e3:.2f} ms/sample", flush=True)
        assert err < 0.6 and err < base_copy
        assert sur_s < solver_s
        sur = surrogate.Surrogate(net, y_scale, solver, solver.lx, solver.ly)
        bad = [(6.0, 3000.0, 3000.0, 2500.0, 10.0)]
        assert not surrogate.in_range(bad, solver.lx, solver.ly)
        out, used = sur.predict([src[21], bad])
        assert used.tolist() == [False, True]
        Hb, _ = solver.run([bad])
        assert np.array_equal(out[1], Hb[0])
        assert not np.array_equal(out[0], H[21])
    finally:
        solver.close()
