"""End to end: solver-generated data, surrogate training on the BF16 kernels,
and what the trained network gains over running the solver.

A small instance of the pipeline (6 x 6 x 3 cubes of 1 km, order 3, eta on a
16 x 16 x 8 grid over 8 s): the trained network must beat the trivial
prediction eta = 0 (relative L2 = 1) on runs it has not seen, and answer
faster per sample than the solver.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_surrogate_learns_and_is_faster_than_the_solver():
    import time
    import torch
    from paper_2107_06640_amd import surrogate
    U, H, solver_s, meta = surrogate.generate(20, grid=16, nt=8, t_end=8.0, order=3, scale=4, log=print)
    assert np.isfinite(H).all() and np.abs(H).max() > 0
    net, hist, scale, X, Y = surrogate.train(U, H, n_train=16, n_val=0, width=8, modes=3, layers=2, hidden=16,
                                             steps=200, batch=16, lr=3e-3, log=print)
    err = surrogate.evaluate(net, X, Y, range(16, 20))
    sel = torch.arange(16, 20, device="cuda:0")
    xb = X[:, sel].contiguous()
    net.forward(xb)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    net.forward(xb)
    torch.cuda.synchronize()
    sur_s = (time.perf_counter() - t0) / 4
    print(f"held-out relative L2 {err:.3f}; solver {solver_s:.3f} s/run, surrogate {sur_s * 1e3:.2f} ms/sample")
    assert err < 0.6
    assert sur_s < solver_s
