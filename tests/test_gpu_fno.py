"""Surrogate kernels on the GPU against their definitions and the FP64 oracle.

* fno_gemm: operands rounded to BF16 (nearest even) then multiplied exactly
  (FP64 on the host): the kernel may differ only by FP32 accumulation,
  bounded here by 1e-5 of sum |a||b|.
* elementwise kernels: their formulas in FP64 (GELU via erf), 1e-5.
* whole network, forward and every parameter gradient: against the FP64
  oracle; BF16 operands give about 2^-9 relative error per product. The
  forward value passes about ten rounded products per layer (3e-2 of the
  largest value); a gradient passes those of the forward and the backward
  chain and is summed over all points (5e-2).
* a few Adam steps on a fixed batch lower the loss.
"""
import math

import numpy as np
import pytest
import torch

from oracle import fno as ofno

pytestmark = pytest.mark.gpu


def bf16(x):
    return torch.as_tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64)


def kernels():
    from paper_2107_06640_amd.fno import Kernels
    return Kernels()


def dev(x):
    return torch.tensor(np.asarray(x), dtype=torch.float32, device="cuda:0").contiguous()


@pytest.mark.parametrize("case", [
    # batch, M, N, K, transA, transB, split, beta
    (1, 70, 45, 33, False, False, 1, 0.0),
    (3, 64, 64, 64, True, False, 1, 1.0),
    (5, 17, 130, 100, False, True, 1, -0.5),
    (2, 129, 31, 4000, True, True, 7, 0.0),
    (1, 32, 32, 100000, False, True, 64, 0.0),
])
def test_gemm_matches_bf16_rounded_product(case):
    batch, M, N, K, ta, tb, split, beta = case
    rng = np.random.default_rng(batch * 1000 + M)
    a = rng.standard_normal((batch, M, K))
    b = rng.standard_normal((batch, K, N))
    c0 = rng.standard_normal((batch, M, N))
    A = dev(np.ascontiguousarray(a.transpose(0, 2, 1)) if ta else a)
    B = dev(np.ascontiguousarray(b.transpose(0, 2, 1)) if tb else b)
    Cd = dev(c0)
    sAm, sAk = (1, M) if ta else (K, 1)
    sBk, sBn = (1, K) if tb else (N, 1)
    k = kernels()
    k.gemm(batch, M, N, K, 1.5, A, 0, M * K, sAm, sAk, B, 0, K * N, sBk, sBn, beta, Cd, 0, M * N, N, 1, split)
    torch.cuda.synchronize()
    want = 1.5 * torch.bmm(bf16(a), bf16(b)) + beta * torch.tensor(c0, dtype=torch.float64).float().double()
    bound = 1.5 * torch.bmm(bf16(a).abs(), bf16(b).abs()) + abs(beta) * np.abs(c0)
    err = (Cd.cpu().double() - want).abs()
    assert (err <= 1e-5 * bound + 1e-6).all(), float((err / (bound + 1e-30)).max())


def test_elementwise_kernels():
    rng = np.random.default_rng(4)
    k = kernels()
    Cc, S, n_outer = 5, 777, 3
    z = rng.standard_normal((n_outer, Cc, S)) * 2
    bias = rng.standard_normal(Cc)
    zd, bd = dev(z), dev(bias)
    a = torch.empty_like(zd)
    k.bias_act(n_outer, Cc, S, zd, bd, a, True)
    zb = z + bias[None, :, None]
    gelu = 0.5 * zb * (1 + np.vectorize(math.erf)(zb / math.sqrt(2)))
    torch.cuda.synchronize()
    assert np.abs(zd.cpu().numpy() - zb).max() < 1e-5
    assert np.abs(a.cpu().numpy() - gelu).max() < 1e-5
    da = rng.standard_normal(z.shape)
    dz = torch.empty_like(zd)
    k.gelu_backward(zd, dev(da), dz)
    phi = np.exp(-0.5 * zb * zb) / math.sqrt(2 * math.pi)
    want = da * (0.5 * (1 + np.vectorize(math.erf)(zb / math.sqrt(2))) + zb * phi)
    torch.cuda.synchronize()
    assert np.abs(dz.cpu().numpy() - want).max() < 1e-5 * np.abs(want).max() + 1e-6
    db = torch.empty(Cc, device="cuda:0")
    k.channel_sum(n_outer, Cc, S, dev(da), db)
    torch.cuda.synchronize()
    assert np.abs(db.cpu().numpy() - da.sum(axis=(0, 2))).max() < 1e-4
    p, g = rng.standard_normal(1000), rng.standard_normal(1000)
    m, v = rng.standard_normal(1000) * 0.1, np.abs(rng.standard_normal(1000)) * 0.1
    pd, md, vd = dev(p), dev(m), dev(v)
    k.adam(pd, dev(g), md, vd, 1e-3, 0.9, 0.999, 1e-8, 7)
    pw, mw, vw = ofno.adam(p, g, m, v, 1e-3, 0.9, 0.999, 1e-8, 7)
    torch.cuda.synchronize()
    assert np.abs(pd.cpu().numpy() - pw).max() < 1e-6 and np.abs(md.cpu().numpy() - mw).max() < 1e-6
    Bn, n = 4, 3000
    yh, y = rng.standard_normal((Bn, n)), rng.standard_normal((Bn, n))
    loss = torch.empty(Bn + 1, device="cuda:0")
    gr = torch.empty(Bn * n, device="cuda:0")
    k.rel_l2(Bn, n, dev(yh), dev(y), loss, gr)
    per = np.linalg.norm(yh - y, axis=1) / np.linalg.norm(y, axis=1)
    gw = (yh - y) / (np.linalg.norm(yh - y, axis=1) * np.linalg.norm(y, axis=1))[:, None] / Bn
    torch.cuda.synchronize()
    assert abs(float(loss[0]) - per.mean()) < 1e-5 and np.abs(loss[1:].cpu().numpy() - per).max() < 1e-5
    assert np.abs(gr.cpu().numpy().reshape(Bn, n) - gw).max() < 1e-5 * np.abs(gw).max()


def small_net(X=16, Y=12, T=8, m=3, B=3, seed=5):
    from paper_2107_06640_amd.fno import FNO
    net = FNO(X, Y, T, cin=3, width=8, modes=m, layers=3, hidden=16, seed=seed)
    rng = np.random.default_rng(seed)
    u = rng.standard_normal((3, B, X, Y, T))
    y = rng.standard_normal((1, B, X, Y, T))
    return net, u, y


def test_network_forward_backward_against_oracle():
    net, u, y = small_net()
    p = net.numpy_params()
    yhat = net.forward(dev(u), keep=True)
    loss, grad = net.loss(yhat, dev(y))
    net.backward(grad)
    torch.cuda.synchronize()
    ref_loss, ref_y, ref_g = ofno.loss_and_grads(p, u, y, net.m, net.L)
    e = np.abs(yhat.cpu().numpy() - ref_y).max() / np.abs(ref_y).max()
    print("forward rel err", e, "loss", float(loss[0]), ref_loss)
    assert e < 3e-2
    assert abs(float(loss[0]) - ref_loss) < 3e-2 * ref_loss
    for name, g in ref_g.items():
        got = net.grads[name].cpu().numpy()
        rel = np.abs(got - g).max() / max(np.abs(g).max(), 1e-30)
        print(name, "grad rel err", rel)
        assert rel < 5e-2, name


def test_adam_training_lowers_the_loss():
    net, u, y = small_net(seed=8)
    ud, yd = dev(u), dev(0.3 * u[:1] + 0.1 * u[1:2] ** 2)
    losses = []
    for _ in range(40):
        yhat = net.forward(ud, keep=True)
        loss, grad = net.loss(yhat, yd)
        net.backward(grad)
        net.adam_step(lr=3e-3)
        losses.append(float(loss[0]))
    print("loss", losses[0], "->", losses[-1])
    assert losses[-1] < 0.5 * losses[0]
