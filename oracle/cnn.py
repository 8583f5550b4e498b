"""Oracle for the learned warm start: a small 3-D convolution network (FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper has no learned component; the network follows the warm-start
description this build implements: five 3x3x3 convolutions with circular
(periodic) padding, widths 1 -> C -> C -> C -> C -> 1, bias on every layer,
exact GELU u/2 (1 + erf(u/sqrt 2)) after the first four.  Input x is the
source term scaled to unit standard deviation, x = f h^2 / s with
s = std(f h^2); the output y scales back to a potential phi0 = s y.

Arrays: a field with C channels is [C, n, n, n] indexed (channel, x, y, z);
weights are w[o, c, 1+dx, 1+dy, 1+dz] for the tap that reads the input at
offset (dx, dy, dz): y[o, p] = b[o] + sum_{c, d} w[o, c, d] x[c, p + d].

``quantize=True`` rounds weights, the network input and every stored
activation to bfloat16 (round to nearest even) at the points where the GPU
stores them, while doing the arithmetic in FP64; that is the reference the
GPU's BF16 kernels (FP32 accumulation) are compared with.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

__all__ = ["bf16_round", "conv3d", "conv3d_adjoint_input", "conv3d_weight_grad", "gelu", "gelu_grad",
           "init_params", "forward", "backward", "adam_step", "loss_mse"]

TAPS = [(dx, dy, dz) for dx in (-1, 0, 1) for dy in (-1, 0, 1) for dz in (-1, 0, 1)]


def bf16_round(a: np.ndarray) -> np.ndarray:
    """Round to the nearest bfloat16 (8-bit significand), ties to even, returned as float64.

    The value is first rounded to float32 (as a GPU would hold it) and then its
    low 16 bits are rounded away.
    """
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    u = (u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def shift(x: np.ndarray, d: tuple[int, int, int]) -> np.ndarray:
    """out[..., p] = x[..., p + d] with periodic wrap (spatial axes are the last three)."""
    return np.roll(x, shift=(-d[0], -d[1], -d[2]), axis=(-3, -2, -1))


def conv3d(x: np.ndarray, w: np.ndarray, b: np.ndarray | None) -> np.ndarray:
    """Circular 3x3x3 convolution (cross-correlation), [C,n,n,n] -> [O,n,n,n]."""
    O = w.shape[0]
    y = np.zeros((O,) + x.shape[1:])
    for d in TAPS:
        xs = shift(x, d)
        y += np.einsum("oc,cxyz->oxyz", w[:, :, d[0] + 1, d[1] + 1, d[2] + 1], xs)
    if b is not None:
        y += b[:, None, None, None]
    return y


def conv3d_adjoint_input(dy: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Gradient of conv3d with respect to its input: dx[c, q] = sum_{o, d} w[o, c, d] dy[o, q - d]."""
    C = w.shape[1]
    dx = np.zeros((C,) + dy.shape[1:])
    for d in TAPS:
        dys = shift(dy, (-d[0], -d[1], -d[2]))
        dx += np.einsum("oc,oxyz->cxyz", w[:, :, d[0] + 1, d[1] + 1, d[2] + 1], dys)
    return dx


def conv3d_weight_grad(x: np.ndarray, dy: np.ndarray) -> np.ndarray:
    """dw[o, c, d] = sum_p dy[o, p] x[c, p + d]."""
    O, C = dy.shape[0], x.shape[0]
    dw = np.zeros((O, C, 3, 3, 3))
    for d in TAPS:
        dw[:, :, d[0] + 1, d[1] + 1, d[2] + 1] = np.einsum("oxyz,cxyz->oc", dy, shift(x, d))
    return dw


def gelu(u: np.ndarray) -> np.ndarray:
    return 0.5 * u * (1.0 + erf(u / math.sqrt(2.0)))


def gelu_grad(u: np.ndarray) -> np.ndarray:
    """d/du [u Phi(u)] = Phi(u) + u phi(u)."""
    return 0.5 * (1.0 + erf(u / math.sqrt(2.0))) + u * np.exp(-0.5 * u * u) / math.sqrt(2.0 * math.pi)


def init_params(channels: int = 24, layers: int = 5, seed: int = 0):
    """He-style normal initialisation; returns a list of (w, b)."""
    rng = np.random.default_rng(seed)
    widths = [1] + [channels] * (layers - 1) + [1]
    params = []
    for l in range(layers):
        ci, co = widths[l], widths[l + 1]
        std = math.sqrt(2.0 / (27 * ci))
        params.append((rng.standard_normal((co, ci, 3, 3, 3)) * std, np.zeros(co)))
    return params


def forward(x: np.ndarray, params, quantize: bool = False):
    """x: [n,n,n] -> (y [n,n,n], cache).  GELU after every layer except the last."""
    q = bf16_round if quantize else (lambda a: a)
    a = q(np.asarray(x, dtype=np.float64))[None]
    cache = []
    L = len(params)
    for l, (w, b) in enumerate(params):
        z = conv3d(a, q(w), b)
        if l < L - 1:
            zq = q(z)
            cache.append((a, zq))
            a = q(gelu(zq))
        else:
            cache.append((a, None))
            return z[0], cache
    raise AssertionError


def backward(dy: np.ndarray, params, cache, quantize: bool = False):
    """Returns ([(dw, db)] per layer, dx [n,n,n]) for upstream gradient dy = dL/dy."""
    q = bf16_round if quantize else (lambda a: a)
    grads = [None] * len(params)
    g = np.asarray(dy, dtype=np.float64)[None]          # dL/dz of the last layer
    for l in range(len(params) - 1, -1, -1):
        w, _ = params[l]
        a_in, _ = cache[l]
        grads[l] = (conv3d_weight_grad(a_in, g), g.sum(axis=(1, 2, 3)))
        da = conv3d_adjoint_input(g, q(w))
        if l > 0:
            _, z_prev = cache[l - 1]
            g = q(da * gelu_grad(z_prev))
        else:
            return grads, da[0]
    raise AssertionError


def loss_mse(y: np.ndarray, t: np.ndarray) -> tuple[float, np.ndarray]:
    """Mean squared error and its gradient with respect to y."""
    r = np.asarray(y, dtype=np.float64) - t
    return float(np.mean(r * r)), 2.0 * r / r.size


def adam_step(p: np.ndarray, g: np.ndarray, m: np.ndarray, v: np.ndarray, t: int, lr: float,
              b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam update (bias-corrected); returns new (p, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
