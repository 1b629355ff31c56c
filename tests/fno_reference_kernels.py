"""CPU stand-in for the surrogate's kernel interface (test helper).

Implements the calls of paper_2107_06640_amd.fno.Kernels with torch CPU
tensors in the tensors' own precision (float64 in the tests), reading and
writing through the same strides and offsets the network code (fno.py) passes, and checking
that every strided view stays inside its tensor. It lets the CPU tests check
the network's composition of products (its layouts and strides) against the
FFT-based oracle before any kernel runs on a GPU.
"""
import torch


def _view(t, off, batch, rows, cols, sb, sr, sc):
    n = t.numel()
    if min(batch, rows, cols) <= 0:
        return None
    last = off + (batch - 1) * sb + (rows - 1) * sr + (cols - 1) * sc
    assert off >= 0 and 0 <= last < n and min(sb, sr, sc) >= 0, (off, last, n)
    return torch.as_strided(t.view(-1), (batch, rows, cols), (sb, sr, sc), off)


class ReferenceKernels:
    def __init__(self):
        self.calls = 0

    def gemm(self, batch, M, N, K, alpha, A, a_off, sAb, sAm, sAk, B, b_off, sBb, sBk, sBn, beta, Cc, c_off,
             sCb, sCm, sCn, split_k=1):
        self.calls += 1
        a = _view(A, a_off, batch, M, K, sAb, sAm, sAk)
        b = _view(B, b_off, batch, K, N, sBb, sBk, sBn)
        c = _view(Cc, c_off, batch, M, N, sCb, sCm, sCn)
        prod = torch.bmm(a.contiguous(), b.contiguous())
        new = alpha * prod + (beta * c if beta != 0.0 else 0.0)
        c.copy_(new)

    def bias_act(self, n_outer, C, S, z, bias, a, act):
        zz = z.view(n_outer, C, S)
        if bias is not None:
            zz += bias.view(1, C, 1)
        out = torch.nn.functional.gelu(zz) if act else zz.clone()
        a.view(n_outer, C, S).copy_(out)

    def gelu_backward(self, z, da, dz):
        x = z.detach().clone().requires_grad_(True)
        y = torch.nn.functional.gelu(x)
        (g,) = torch.autograd.grad(y, x, da)
        dz.copy_(g)

    def channel_sum(self, n_outer, C, S, dz, db):
        db.copy_(dz.view(n_outer, C, S).sum(dim=(0, 2)))

    def adam(self, p, g, m, v, lr, b1, b2, eps, t):
        m.mul_(b1).add_((1 - b1) * g)
        v.mul_(b2).add_((1 - b2) * g * g)
        p.sub_(lr * (m / (1 - b1 ** t)) / (torch.sqrt(v / (1 - b2 ** t)) + eps))

    def rel_l2(self, n_batch, n, yhat, y, loss, grad):
        d = (yhat - y).view(n_batch, n)
        ne = d.norm(dim=1)
        ny = y.view(n_batch, n).norm(dim=1)
        loss[1:] = ne / ny
        loss[0] = (ne / ny).mean()
        if grad is not None:
            grad.view(n_batch, n).copy_(d / (ne * ny)[:, None] / n_batch)

    def scale(self, x, s):
        x.mul_(s)
