"""Spectral neural-operator surrogate on the library's BF16 matrix-core kernels.

Maps a seafloor uplift field to the sea-surface height eta(x, y, t). The
network (a Fourier neural operator):

    v0 = P u + p                                  pointwise lift, Cin -> W channels
    v_{l+1} = act(K_l v_l + W_l v_l + b_l)        l < L; act = GELU except after the last layer
    h = GELU(Q1 v_L + q1), y = Q2 h + q2          pointwise projection W -> H -> 1

K_l is the spectral convolution: real FFT over (x, y, t), keep the modes
kx, ky in {0..m-1} and {n-m..n-1} and kt in {0..m-1}, multiply each kept mode
by a complex W x W matrix, inverse real FFT. Here the transforms are dense
DFT matrices, so every step is a matrix product on fno_gemm (include/fno.h);
this module only lays out memory and sequences the calls (torch tensors are
device memory). Activations are channel-major: [C][batch][X][Y][T], so that
every pointwise product and every transform stage is one strided product.
"""
from __future__ import annotations

import ctypes as C
import math

import numpy as np

from . import seis as _seis


def _lib():
    lib = _seis.load_library()
    if not getattr(lib, "_fno_declared", False):
        i64, f32, P = C.c_int64, C.c_float, C.c_void_p
        lib.fno_gemm.argtypes = [i64, i64, i64, i64, f32, P, i64, i64, i64, P, i64, i64, i64, f32, P, i64, i64, i64,
                                 C.c_int, P]
        lib.fno_bias_act.argtypes = [i64, i64, i64, P, P, P, C.c_int, P]
        lib.fno_gelu_backward.argtypes = [i64, P, P, P, P]
        lib.fno_channel_sum.argtypes = [i64, i64, i64, P, P, P]
        lib.fno_adam.argtypes = [i64, P, P, P, P, f32, f32, f32, f32, C.c_int, P]
        lib.fno_rel_l2.argtypes = [i64, i64, P, P, P, P, P]
        lib.fno_scale.argtypes = [i64, P, f32, P]
        for n in ("fno_gemm", "fno_bias_act", "fno_gelu_backward", "fno_channel_sum", "fno_adam", "fno_rel_l2",
                  "fno_scale"):
            getattr(lib, n).restype = C.c_int
        lib._fno_declared = True
    return lib


def _chk(rc, what):
    if rc != 0:
        raise RuntimeError(f"{what} failed with code {rc}")


def _p(t):
    return None if t is None else C.c_void_p(t.data_ptr())


class Kernels:
    """Thin wrappers of the C ABI on torch device tensors (float32, contiguous)."""

    def __init__(self, stream=None):
        self.lib = _lib()
        self.stream = None if stream is None else C.c_void_p(stream)

    def gemm(self, batch, M, N, K, alpha, A, a_off, sAb, sAm, sAk, B, b_off, sBb, sBk, sBn, beta, Cc, c_off,
             sCb, sCm, sCn, split_k=1):
        """C = alpha A B + beta C on strided views (offsets in elements)."""
        pa = C.c_void_p(A.data_ptr() + 4 * a_off)
        pb = C.c_void_p(B.data_ptr() + 4 * b_off)
        pc = C.c_void_p(Cc.data_ptr() + 4 * c_off)
        _chk(self.lib.fno_gemm(batch, M, N, K, alpha, pa, sAb, sAm, sAk, pb, sBb, sBk, sBn, beta, pc, sCb, sCm, sCn,
                               split_k, self.stream), "fno_gemm")

    def bias_act(self, n_outer, Cc, S, z, bias, a, act):
        _chk(self.lib.fno_bias_act(n_outer, Cc, S, _p(z), _p(bias), _p(a), 1 if act else 0, self.stream),
             "fno_bias_act")

    def gelu_backward(self, z, da, dz):
        _chk(self.lib.fno_gelu_backward(z.numel(), _p(z), _p(da), _p(dz), self.stream), "fno_gelu_backward")

    def channel_sum(self, n_outer, Cc, S, dz, db):
        _chk(self.lib.fno_channel_sum(n_outer, Cc, S, _p(dz), _p(db), self.stream), "fno_channel_sum")

    def adam(self, p, g, m, v, lr, b1, b2, eps, t):
        _chk(self.lib.fno_adam(p.numel(), _p(p), _p(g), _p(m), _p(v), lr, b1, b2, eps, t, self.stream), "fno_adam")

    def rel_l2(self, n_batch, n, yhat, y, loss, grad):
        _chk(self.lib.fno_rel_l2(n_batch, n, _p(yhat), _p(y), _p(loss), _p(grad), self.stream), "fno_rel_l2")

    def scale(self, x, s):
        _chk(self.lib.fno_scale(x.numel(), _p(x), s, self.stream), "fno_scale")


def mode_indices(n, m):
    """Kept frequencies of a full DFT axis of length n: 0..m-1 and n-m..n-1."""
    return np.concatenate([np.arange(m), np.arange(n - m, n)])


def dft_matrices(X, Y, T, m):
    """Dense forward and inverse DFT factors (float64), numpy's rfftn/irfftn conventions.

    Forward (unnormalised): along t a real signal gives kt < m (re | im);
    along y and x complex signals give the kept modes (re | im).
    Inverse: 1/n per axis; the t axis is a real inverse with weight 1 for
    kt = 0 and 2 for kt > 0 (Hermitian half spectrum, imaginary part of kt = 0
    dropped).
    """
    out = {}
    t = np.arange(T)
    kt = np.arange(m)
    th = 2 * np.pi * np.outer(t, kt) / T                   # [T, m]
    out["Ft"] = np.concatenate([np.cos(th), -np.sin(th)], axis=1)      # [T, 2m]: (p, kt)
    ck = np.where(kt == 0, 1.0, 2.0) / T
    out["Gt"] = np.concatenate([(ck * np.cos(th)).T, (-ck * np.sin(th)).T], axis=0)  # [2m, T]
    for name, n in (("y", Y), ("x", X)):
        k = mode_indices(n, m)
        j = np.arange(n)
        ph = 2 * np.pi * np.outer(k, j) / n                 # [2m, n]
        c, s = np.cos(ph), np.sin(ph)
        # forward: (a + ib) e^{-i ph}: re = a c + b s, im = b c - a s
        out[f"F{name}_re"] = np.concatenate([c, -s], axis=0)  # multiplies a, rows (q, k)
        out[f"F{name}_im"] = np.concatenate([s, c], axis=0)   # multiplies b
        # inverse: (1/n) sum_k (a + ib) e^{+i ph}: re = (a c - b s)/n, im = (a s + b c)/n
        out[f"G{name}_re"] = np.concatenate([c.T, -s.T], axis=1) / n   # [n, (r, k)] -> real part
        out[f"G{name}_im"] = np.concatenate([s.T, c.T], axis=1) / n    # -> imaginary part
    return out


class FNO:
    """Parameters, forward and backward of the operator network on one device.

    shapes: input [Cin][B][X][Y][T], output [1][B][X][Y][T], float32 tensors on
    the device. Parameters are FP32 masters; the products round them to BF16.
    """

    def __init__(self, X, Y, T, cin=4, width=32, modes=12, layers=4, hidden=128, seed=0, device="cuda:0",
                 stream=None, kernels=None, dtype=None):
        import torch
        self.torch = torch
        self.dtype = torch.float32 if dtype is None else dtype
        self.X, self.Y, self.T, self.cin, self.W, self.m, self.L, self.H = X, Y, T, cin, width, modes, layers, hidden
        self.dev = device
        self.k = Kernels(stream) if kernels is None else kernels
        self.nm = (2 * modes) * (2 * modes) * modes
        rng = np.random.default_rng(seed)
        W, m = width, modes

        def dense(o, i):
            return rng.uniform(-1, 1, (o, i)) / math.sqrt(i)

        scale = 1.0 / (W * W)
        p = {"P": dense(W, cin), "p": np.zeros(W)}
        for l in range(layers):
            p[f"W{l}"] = dense(W, W)
            p[f"b{l}"] = np.zeros(W)
            p[f"R{l}"] = scale * rng.uniform(0, 1, (2, self.nm, W, W))   # [re|im][mode][ci][co]
        p["Q1"] = dense(hidden, W)
        p["q1"] = np.zeros(hidden)
        p["Q2"] = dense(1, hidden)
        p["q2"] = np.zeros(1)
        self.names = list(p)
        self.params = {k: torch.tensor(v, dtype=self.dtype, device=device).contiguous() for k, v in p.items()}
        self.grads = {k: torch.zeros_like(v) for k, v in self.params.items()}
        self.adam_m = {k: torch.zeros_like(v) for k, v in self.params.items()}
        self.adam_v = {k: torch.zeros_like(v) for k, v in self.params.items()}
        self.step_count = 0
        self.mats = {k: torch.tensor(v, dtype=self.dtype, device=device).contiguous()
                     for k, v in dft_matrices(X, Y, T, modes).items()}

    # -- parameters as float64 numpy (for the oracle and checkpoints)
    def numpy_params(self):
        return {k: v.detach().cpu().double().numpy() for k, v in self.params.items()}

    def load_numpy_params(self, p):
        for k, v in p.items():
            self.params[k].copy_(self.torch.tensor(v, dtype=self.dtype))

    # ------------------------------------------------------------------
    def _empty(self, *shape):
        return self.torch.empty(*shape, dtype=self.dtype, device=self.dev)

    def _pointwise(self, Wm, x, z, cin, cout, n, beta=0.0):
        """z[cout][n] = Wm[cout][cin] x[cin][n] (+ beta z)."""
        self.k.gemm(1, cout, n, cin, 1.0, Wm, 0, 0, cin, 1, x, 0, 0, n, 1, beta, z, 0, 0, n, 1)

    def _spectral_forward(self, R, v, B, out):
        """out += K v (out already holds W v); returns the kept modes of v (for the weight gradient)."""
        X, Y, T, W, m, nm = self.X, self.Y, self.T, self.W, self.m, self.nm
        k, M = self.k, self.mats
        m2 = 2 * m
        rows = W * B * X * Y
        U1 = self._empty(rows * m2)                        # [(c,b,x,y)][(p,kt)]
        k.gemm(1, rows, m2, T, 1.0, v, 0, 0, T, 1, M["Ft"], 0, 0, m2, 1, 0.0, U1, 0, 0, m2, 1)
        nb = W * B * X
        U2 = self._empty(nb * 2 * m2 * m)                  # [(c,b,x)][(q,ky)][kt]
        for pi, F in ((0, M["Fy_re"]), (1, M["Fy_im"])):
            k.gemm(nb, 2 * m2, m, Y, 1.0, F, 0, 0, Y, 1, U1, pi * m, Y * m2, m2, 1, float(pi), U2, 0, 2 * m2 * m, m, 1)
        nc = W * B
        inner = m2 * m                                     # (ky, kt) per part
        U3 = self._empty(nc * 2 * m2 * inner)              # [(c,b)][(r,kx)][(ky,kt)] = [c][b][r][mode]
        for pi, F in ((0, M["Fx_re"]), (1, M["Fx_im"])):
            k.gemm(nc, 2 * m2, inner, X, 1.0, F, 0, 0, X, 1, U2, pi * inner, X * 2 * inner, 2 * inner, 1, float(pi),
                   U3, 0, 2 * m2 * inner, inner, 1)
        # per-mode complex channel mixing: Y[co][b][r][mode] = sum_ci U3[ci][b][.][mode] R[.][mode][ci][co]
        Ym = self._empty(W * B * 2 * nm)
        sC, sB_ = B * 2 * nm, 2 * nm                       # channel and batch strides of U3 / Ym
        Rre, Rim = 0, nm * W * W
        terms = ((0, 0, Rre, 1.0, 0.0), (0, nm, Rim, -1.0, 1.0), (nm, 0, Rim, 1.0, 0.0), (nm, nm, Rre, 1.0, 1.0))
        for (yo, io, ro, alpha, beta) in terms:
            k.gemm(nm, B, W, W, alpha, U3, io, 1, sB_, sC, R, ro, W * W, W, 1, beta, Ym, yo, 1, sB_, sC)
        # inverse along x: V2[(c,b)][x][(q, ky, kt)]
        V2 = self._empty(nc * X * 2 * inner)
        for qi, G in ((0, M["Gx_re"]), (1, M["Gx_im"])):
            k.gemm(nc, X, inner, 2 * m2, 1.0, G, 0, 0, 2 * m2, 1, Ym, 0, 2 * nm, inner, 1, 0.0, V2, qi * inner,
                   X * 2 * inner, 2 * inner, 1)
        # inverse along y: V1[(c,b,x)][y][(p, kt)]
        V1 = self._empty(nb * Y * m2)
        for qi, G in ((0, M["Gy_re"]), (1, M["Gy_im"])):
            k.gemm(nb, Y, m, 2 * m2, 1.0, G, 0, 0, 2 * m2, 1, V2, 0, 2 * inner, m, 1, 0.0, V1, qi * m, Y * m2, m2, 1)
        # inverse real transform along t, added to out
        k.gemm(1, rows, T, m2, 1.0, V1, 0, 0, m2, 1, M["Gt"], 0, 0, T, 1, 1.0, out, 0, 0, T, 1)
        return U3

    def _spectral_backward(self, R, U3, dout, B, dv, dR):
        """dv += K^T dout; dR = gradient of the mixing weights."""
        X, Y, T, W, m, nm = self.X, self.Y, self.T, self.W, self.m, self.nm
        k, M = self.k, self.mats
        m2 = 2 * m
        rows = W * B * X * Y
        nb, nc, inner = W * B * X, W * B, m2 * m
        dV1 = self._empty(rows * m2)
        k.gemm(1, rows, m2, T, 1.0, dout, 0, 0, T, 1, M["Gt"], 0, 0, 1, T, 0.0, dV1, 0, 0, m2, 1)
        dV2 = self._empty(nb * 2 * m2 * m)
        for qi, G in ((0, M["Gy_re"]), (1, M["Gy_im"])):
            # dV2[(q,ky)][kt] += sum_y G[y][(q,ky)] dV1[y][qi*m + kt]
            k.gemm(nb, 2 * m2, m, Y, 1.0, G, 0, 0, 1, 2 * m2, dV1, qi * m, Y * m2, m2, 1, float(qi), dV2, 0,
                   2 * m2 * m, m, 1)
        dYm = self._empty(W * B * 2 * nm)
        for qi, G in ((0, M["Gx_re"]), (1, M["Gx_im"])):
            k.gemm(nc, 2 * m2, inner, X, 1.0, G, 0, 0, 1, 2 * m2, dV2, qi * inner, X * 2 * inner, 2 * inner, 1,
                   float(qi), dYm, 0, 2 * nm, inner, 1)
        sC, sB_ = B * 2 * nm, 2 * nm
        Rre, Rim = 0, nm * W * W
        # dIn_re = R_re dY_re + R_im dY_im ; dIn_im = -R_im dY_re + R_re dY_im  (sums over co)
        dU3 = self._empty(W * B * 2 * nm)
        terms = ((0, 0, Rre, 1.0, 0.0), (0, nm, Rim, 1.0, 1.0), (nm, 0, Rim, -1.0, 0.0), (nm, nm, Rre, 1.0, 1.0))
        for (io, yo, ro, alpha, beta) in terms:
            k.gemm(nm, B, W, W, alpha, dYm, yo, 1, sB_, sC, R, ro, W * W, 1, W, beta, dU3, io, 1, sB_, sC)
        # dR_re = sum_b In_re dY_re + In_im dY_im ; dR_im = sum_b In_re dY_im - In_im dY_re
        wterms = ((Rre, 0, 0, 1.0, 0.0), (Rre, nm, nm, 1.0, 1.0), (Rim, 0, nm, 1.0, 0.0), (Rim, nm, 0, -1.0, 1.0))
        for (ro, io, yo, alpha, beta) in wterms:
            k.gemm(nm, W, W, B, alpha, U3, io, 1, sC, sB_, dYm, yo, 1, sB_, sC, beta, dR, ro, W * W, W, 1)
        # back through the forward transforms
        dU2 = self._empty(nc * X * 2 * inner)
        for pi, F in ((0, M["Fx_re"]), (1, M["Fx_im"])):
            k.gemm(nc, X, inner, 2 * m2, 1.0, F, 0, 0, 1, X, dU3, 0, 2 * nm, inner, 1, 0.0, dU2, pi * inner,
                   X * 2 * inner, 2 * inner, 1)
        dU1 = self._empty(rows * m2)
        for pi, F in ((0, M["Fy_re"]), (1, M["Fy_im"])):
            k.gemm(nb, Y, m, 2 * m2, 1.0, F, 0, 0, 1, Y, dU2, 0, 2 * m2 * m, m, 1, 0.0, dU1, pi * m, Y * m2, m2, 1)
        k.gemm(1, rows, T, m2, 1.0, dU1, 0, 0, m2, 1, M["Ft"], 0, 0, 1, m2, 1.0, dv, 0, 0, T, 1)

    # ------------------------------------------------------------------
    def forward(self, u, keep=False):
        """u: [Cin][B][X][Y][T] device tensor -> y [1][B][X][Y][T]."""
        B = u.shape[1]
        S = B * self.X * self.Y * self.T
        W, k, P = self.W, self.k, self.params
        tape = {"u": u}
        v = self._empty(W * S)
        self._pointwise(P["P"], u, v, self.cin, W, S)
        k.bias_act(1, W, S, v, P["p"], v, False)
        for l in range(self.L):
            z = self._empty(W * S)
            self._pointwise(P[f"W{l}"], v, z, W, W, S)
            U3 = self._spectral_forward(P[f"R{l}"], v, B, z)
            last = l == self.L - 1
            a = self._empty(W * S) if not last else z
            k.bias_act(1, W, S, z, P[f"b{l}"], a, not last)
            if keep:
                tape[f"v{l}"], tape[f"z{l}"], tape[f"U{l}"] = v, z, U3
            v = a
        h = self._empty(self.H * S)
        self._pointwise(P["Q1"], v, h, W, self.H, S)
        g = self._empty(self.H * S)
        k.bias_act(1, self.H, S, h, P["q1"], g, True)
        y = self._empty(S)
        self._pointwise(P["Q2"], g, y, self.H, 1, S)
        k.bias_act(1, 1, S, y, P["q2"], y, False)
        if keep:
            tape.update(vL=v, h=h, g=g, B=B)
            self.tape = tape
        return y.view(1, B, self.X, self.Y, self.T)

    def _weight_grad(self, dz, x, dW, cout, cin, n):
        """dW[cout][cin] = sum_n dz[cout][n] x[cin][n] (split over n)."""
        split = max(1, min(4096, n // 8192))
        self.k.gemm(1, cout, cin, n, 1.0, dz, 0, 0, n, 1, x, 0, 0, 1, n, 0.0, dW, 0, 0, cin, 1, split)

    def backward(self, dy):
        """Gradients of all parameters for the output gradient dy [1][B][X][Y][T] (after forward(keep=True))."""
        t, k, P, G = self.tape, self.k, self.params, self.grads
        B = t["B"]
        S = B * self.X * self.Y * self.T
        W, H = self.W, self.H
        dy = dy.reshape(-1).contiguous()
        k.channel_sum(1, 1, S, dy, G["q2"])
        self._weight_grad(dy, t["g"], G["Q2"], 1, H, S)
        dg = self._empty(H * S)
        self._pointwise_t(P["Q2"], dy, dg, 1, H, S)
        k.gelu_backward(t["h"], dg, dg)
        k.channel_sum(1, H, S, dg, G["q1"])
        self._weight_grad(dg, t["vL"], G["Q1"], H, W, S)
        dv = self._empty(W * S)
        self._pointwise_t(P["Q1"], dg, dv, H, W, S)
        del dg
        for l in reversed(range(self.L)):
            last = l == self.L - 1
            dz = dv
            if not last:
                k.gelu_backward(t[f"z{l}"], dv, dz)
            k.channel_sum(1, W, S, dz, G[f"b{l}"])
            v = t[f"v{l}"]
            self._weight_grad(dz, v, G[f"W{l}"], W, W, S)
            dvn = self._empty(W * S)
            self._pointwise_t(P[f"W{l}"], dz, dvn, W, W, S)
            self._spectral_backward(P[f"R{l}"], t[f"U{l}"], dz, B, dvn, G[f"R{l}"])
            dv = dvn
        k.channel_sum(1, W, S, dv, G["p"])
        self._weight_grad(dv, t["u"], G["P"], W, self.cin, S)
        return G

    def _pointwise_t(self, Wm, dz, dx, cout, cin, n):
        """dx[cin][n] = Wm^T dz (Wm is [cout][cin])."""
        self.k.gemm(1, cin, n, cout, 1.0, Wm, 0, 0, 1, cin, dz, 0, 0, n, 1, 0.0, dx, 0, 0, n, 1)

    def loss(self, yhat, y, grad=True):
        """Mean relative L2 over the batch; returns (loss tensor [B+1], gradient or None)."""
        B = yhat.shape[1]
        n = yhat.numel() // B
        out = self._empty(B + 1)
        g = self._empty(yhat.numel()) if grad else None
        self.k.rel_l2(B, n, yhat.reshape(-1), y.reshape(-1), out, g)
        return out, g

    def adam_step(self, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.step_count += 1
        for name in self.names:
            self.k.adam(self.params[name], self.grads[name], self.adam_m[name], self.adam_v[name], lr, b1, b2, eps,
                        self.step_count)


class CountingKernels(Kernels):
    """Kernels that also count the products' algorithmic flops (2 batch M N K per call)
    and bytes (FP32 A and B read once, C read and written once)."""

    def __init__(self, stream=None):
        super().__init__(stream)
        self.flops = 0
        self.bytes = 0
        self.calls = 0

    def gemm(self, batch, M, N, K, *args, **kw):
        self.flops += 2 * batch * M * N * K
        self.bytes += 4 * batch * (M * K + K * N + 2 * M * N)
        self.calls += 1
        super().gemm(batch, M, N, K, *args, **kw)


def bench_main(argv=None):
    """Time training steps of the surrogate's network at its data shape.

        python -m paper_2107_06640_amd.fno [--batch 64] [--steps 5] [--warmup 2]

    A step is forward (kept for the backward), loss, backward and Adam on a
    seeded random batch of the 64 x 64 x 32 grid with 4 input channels
    (width 32, 12 modes, 4 layers, hidden 128). Prints one JSON line: time per
    step and the products' algorithmic flops per step (their rate against
    the BF16 matrix-core peak needs the products' own kernel time, which a
    kernel trace gives).
    """
    import argparse
    import json

    import torch
    ap = argparse.ArgumentParser()
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    a = ap.parse_args(argv)
    torch.cuda.set_device(0)
    k = CountingKernels()
    net = FNO(64, 64, 32, cin=4, width=32, modes=12, layers=4, hidden=128, seed=0, kernels=k)
    g = torch.Generator(device="cuda:0").manual_seed(0)
    u = torch.randn(4, a.batch, 64, 64, 32, device="cuda:0", generator=g)
    y = torch.randn(1, a.batch, 64, 64, 32, device="cuda:0", generator=g)

    def step():
        yhat = net.forward(u, keep=True)
        _, grad = net.loss(yhat, y)
        net.backward(grad)
        net.adam_step()

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    k.flops = k.bytes = k.calls = 0
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(a.steps):
        step()
    t1.record()
    t1.synchronize()
    ms = t0.elapsed_time(t1) / a.steps
    print(json.dumps({"batch": a.batch, "steps": a.steps, "ms_per_step": ms,
                      "gemm_flops_per_step": k.flops / a.steps, "gemm_bytes_per_step": k.bytes / a.steps,
                      "gemm_calls_per_step": k.calls / a.steps,
                      "gemm_tflops_over_step_time": k.flops / a.steps / (ms / 1e3) / 1e12}), flush=True)


if __name__ == "__main__":
    bench_main()
