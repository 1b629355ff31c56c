"""Fourier neural operator: forward, loss and gradients (oracle).

Test infrastructure only (see ``oracle/__init__``). FP64 on the CPU with
plain PyTorch operations: the spectral convolution uses the library FFT
(torch.fft.rfftn / irfftn) and gradients come from automatic
differentiation, which the pins check against finite differences.

Network (the operator of the seafloor-uplift surrogate):
    v0 = P u + p
    v_{l+1} = act(K_l v_l + W_l v_l + b_l), act = GELU (exact erf form) except
              after the last layer
    y = Q2 GELU(Q1 v_L + q1) + q2
K_l: real FFT over (x, y, t); keep kx, ky in {0..m-1} u {n-m..n-1}, kt in
{0..m-1}; out(mode) = sum_ci in_ci(mode) R[ci][co](mode) with R complex;
inverse real FFT of the kept modes (all others zero).
Tensors are channel-major, [C][B][X][Y][T]; R is stored as [2][modes][ci][co]
(real part, imaginary part), modes ordered (kx, ky, kt) with the kept kx and
ky in the order 0..m-1, n-m..n-1.
"""
from __future__ import annotations

import numpy as np
import torch


def kept(n, m):
    return list(range(m)) + list(range(n - m, n))


def spectral(v, R, m):
    """K v for v [C][B][X][Y][T] (torch float64) and R [2][modes][C][C]."""
    Cc, B, X, Y, T = v.shape
    V = torch.fft.rfftn(v, dim=(2, 3, 4))                        # [C][B][X][Y][T//2+1]
    ix = torch.tensor(kept(X, m))
    iy = torch.tensor(kept(Y, m))
    Vk = V[:, :, ix][:, :, :, iy][..., :m]                        # [C][B][2m][2m][m]
    Rc = torch.complex(R[0], R[1]).reshape(2 * m, 2 * m, m, Cc, -1)  # [kx][ky][kt][ci][co]
    Ok = torch.einsum("ibxyt,xytio->obxyt", Vk, Rc)
    O = torch.zeros((Rc.shape[-1], B, X, Y, T // 2 + 1), dtype=V.dtype)
    O[:, :, ix[:, None], iy[None, :], :m] = Ok
    return torch.fft.irfftn(O, s=(X, Y, T), dim=(2, 3, 4))


def pointwise(Wm, v):
    return torch.einsum("oc,cbxyt->obxyt", Wm, v)


def bias(b, v):
    return v + b[:, None, None, None, None]


def forward(params, u, m, layers):
    """params: dict of torch float64 tensors (names as in the library's model)."""
    gelu = torch.nn.functional.gelu
    v = bias(params["p"], pointwise(params["P"], u))
    for l in range(layers):
        z = bias(params[f"b{l}"], pointwise(params[f"W{l}"], v) + spectral(v, params[f"R{l}"], m))
        v = z if l == layers - 1 else gelu(z)
    h = gelu(bias(params["q1"], pointwise(params["Q1"], v)))
    return bias(params["q2"], pointwise(params["Q2"], h))


def rel_l2(yhat, y):
    """Mean over the batch of |yhat_b - y_b| / |y_b| (y, yhat [1][B][...])."""
    B = y.shape[1]
    d = (yhat - y).reshape(B, -1)
    return (d.norm(dim=1) / y.reshape(B, -1).norm(dim=1)).mean()


def loss_and_grads(params_np, u_np, y_np, m, layers):
    """FP64 loss and gradients of every parameter (numpy in, numpy out)."""
    params = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in params_np.items()}
    u = torch.tensor(u_np, dtype=torch.float64)
    y = torch.tensor(y_np, dtype=torch.float64)
    yhat = forward(params, u, m, layers)
    loss = rel_l2(yhat, y)
    loss.backward()
    return float(loss.detach()), yhat.detach().numpy(), {k: v.grad.numpy() for k, v in params.items()}


def predict(params_np, u_np, m, layers):
    with torch.no_grad():
        params = {k: torch.tensor(v, dtype=torch.float64) for k, v in params_np.items()}
        return forward(params, torch.tensor(u_np, dtype=torch.float64), m, layers).numpy()


def adam(p, g, mom, vel, lr, b1, b2, eps, t):
    """One Adam step (Kingma and Ba), returns the new (p, m, v)."""
    mom = b1 * mom + (1 - b1) * g
    vel = b2 * vel + (1 - b2) * g * g
    mh = mom / (1 - b1 ** t)
    vh = vel / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), mom, vel
