"""Learned correction form (oracle).

Test infrastructure only: only tests, the smoke check and the benchmark's CPU
baseline use this module.

The paper's method is the weighted sum of Sec. 2.2 (Eq. "triple_sum") with a
kernel of I points per direction.  The learned form is a variant beside it: a
small network predicts, from the 4 x 4 x 4 stencil the I = 4 Lagrange kernel
uses and from the in-cell offsets, the difference between a wide kernel (the
I = 8 C2 spline of Sec. 2.2 / Appendix "kernels") and the I = 4 Lagrange
interpolant, so that u ~ u_L4 + MLP(features).  The paper does not describe
this form; every choice below is a reading, stated once here:

* Features (195 per particle): the stored FP32 field at the nodes c + i,
  i in {-1, 0, 1, 2} per axis (indices mod N, c from steps 1-3 of Sec. 2.2),
  ordered f = ((k3*4 + k2)*4 + k1)*3 + a with k = i + 1 and a the component,
  then the offsets t1, t2, t3 at f = 192, 193, 194.  Every feature is a BF16
  number: RNE of the FP32 field value, and RNE of fl32(t) for the offsets.
* Target: u_K(X) - u_L4(X) per component, K the wide kernel (FP64 here).
* Network: 195 -> 128 -> 128 -> 3, z1 = W1 x + b1, h1 = silu(z1),
  z2 = W2 h1 + b2, h2 = silu(z2), y = W3 h2 + b3, silu(z) = z / (1 + e^-z).
  Parameters are one FP32 vector in the order W1[128][195], b1[128],
  W2[128][128], b2[128], W3[3][128], b3[3] (41987 numbers).
* Loss: mean over the batch rows and the 3 components of (y - target)^2.
* Optimiser: Adam (Kingma and Ba, 2015) with bias correction, beta1 = 0.9,
  beta2 = 0.999, eps = 1e-8, step size lr0 * (1 + cos(pi * s / S)) / 2 at step
  s of S (cosine decay).  Batches are consecutive slices of the pair arrays in
  their stored order (the pairs come from independent uniform positions, so no
  shuffle is drawn); a trailing partial batch is dropped.
* Reduced precision on the GPU: the two hidden-layer products and the
  backward products through them take BF16 operands (x, W1, h1, W2 forward;
  dz2, h1, W2, dz1, x backward) with FP32 sums; everything else is FP32.
  ``emulate_bf16=True`` rounds exactly those operands to BF16 here (through
  FP32), so that GPU and oracle differ only by summation order and FP32.
* Inference: u = u_L4 + y; an audit runs the wide kernel at every k-th
  particle (k = round(1 / audit_frac), particles 0, k, 2k, ...), and if the
  RMS of (u - u_K) over the audit, relative to the RMS of u_K there, exceeds
  the caller's tolerance, the whole result is replaced by u_K.
"""
from __future__ import annotations

import math

import numpy as np

from . import geometry as G
from . import interp as OI
from . import kernels as K
from .precision import bf16_bits_to_f64, f32_to_bf16_bits

N_IN, N_H, N_OUT = 195, 128, 3
SHAPES = (("W1", (N_H, N_IN)), ("b1", (N_H,)), ("W2", (N_H, N_H)), ("b2", (N_H,)),
          ("W3", (N_OUT, N_H)), ("b3", (N_OUT,)))
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)  # 41987
STENCIL = (-1, 0, 1, 2)


def unpack(params: np.ndarray) -> dict:
    """Views of the flat parameter vector, by name."""
    out, o = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = params[o:o + n].reshape(shape)
        o += n
    return out


def bf16_round(x) -> np.ndarray:
    """RNE to BF16 through FP32, returned as FP64."""
    return bf16_bits_to_f64(f32_to_bf16_bits(np.asarray(x, dtype=np.float64).astype(np.float32)))


def features(field32: np.ndarray, X: np.ndarray) -> np.ndarray:
    """BF16 bits [Np][195] of the stencil values and offsets (see header)."""
    field32 = np.asarray(field32, dtype=np.float32)
    N = field32.shape[0]
    c, t = G.cell_and_offset(np.asarray(X, dtype=np.float64), N)
    Np = c.shape[0]
    out = np.empty((Np, N_IN), dtype=np.uint16)
    f = 0
    for i3 in STENCIL:
        x3 = (c[:, 2] + i3) % N
        for i2 in STENCIL:
            x2 = (c[:, 1] + i2) % N
            for i1 in STENCIL:
                x1 = (c[:, 0] + i1) % N
                vals = field32[x3, x2, x1, :]
                out[:, f:f + 3] = f32_to_bf16_bits(vals)
                f += 3
    out[:, 192:195] = f32_to_bf16_bits(t.astype(np.float32))
    return out


def targets(field: np.ndarray, X: np.ndarray, family: int, I: int, m: int) -> np.ndarray:
    """u_K(X) - u_L4(X), FP64, on the stored field values."""
    wide = OI.interp_vec(field, X, family, I, m)
    narrow = OI.interp_vec(field, X, K.LAGRANGE, 4, 0)
    return wide - narrow


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(params: np.ndarray, x: np.ndarray, emulate_bf16: bool = False):
    """Network output y [B][3] for features x [B][195] (FP64 values), and the
    intermediate arrays the backward pass needs."""
    p = unpack(np.asarray(params, dtype=np.float64))
    r = bf16_round if emulate_bf16 else (lambda a: a)
    x_ = r(x)
    z1 = x_ @ r(p["W1"]).T + p["b1"]
    h1 = silu(z1)
    h1_ = r(h1)
    z2 = h1_ @ r(p["W2"]).T + p["b2"]
    h2 = silu(z2)
    y = h2 @ p["W3"].T + p["b3"]
    return y, (x_, z1, h1, h1_, z2, h2)


def loss_and_grads(params: np.ndarray, x: np.ndarray, target: np.ndarray, emulate_bf16: bool = False):
    """Mean-square loss and its gradient (flat, parameter layout) by the chain rule."""
    p = unpack(np.asarray(params, dtype=np.float64))
    r = bf16_round if emulate_bf16 else (lambda a: a)
    y, (x_, z1, h1, h1_, z2, h2) = forward(params, x, emulate_bf16)
    B = x.shape[0]
    diff = y - target
    loss = float(np.mean(diff * diff))
    dy = 2.0 * diff / (B * N_OUT)
    g = {}
    g["W3"] = dy.T @ h2
    g["b3"] = dy.sum(axis=0)
    dh2 = dy @ p["W3"]
    dz2 = dh2 * dsilu(z2)
    dz2_ = r(dz2)
    g["W2"] = dz2_.T @ h1_
    g["b2"] = dz2.sum(axis=0)
    dh1 = dz2_ @ r(p["W2"])
    dz1 = dh1 * dsilu(z1)
    dz1_ = r(dz1)
    g["W1"] = dz1_.T @ x_
    g["b1"] = dz1.sum(axis=0)
    flat = np.concatenate([g[name].reshape(-1) for name, _ in SHAPES])
    return loss, flat


def cosine_lr(lr0: float, step: int, total: int) -> float:
    return lr0 * 0.5 * (1.0 + math.cos(math.pi * step / total))


def adam_step(params, grads, m, v, step: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counted from 0); returns new (params, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grads
    v = beta2 * v + (1.0 - beta2) * grads * grads
    mh = m / (1.0 - beta1 ** (step + 1))
    vh = v / (1.0 - beta2 ** (step + 1))
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


def train(params0, feats_bits, target, epochs: int, batch: int, lr0: float, emulate_bf16: bool = False):
    """Adam over consecutive batches; returns (params, per-step losses)."""
    x_all = bf16_bits_to_f64(feats_bits)
    n_batches = x_all.shape[0] // batch
    total = epochs * n_batches
    params = np.asarray(params0, dtype=np.float64).copy()
    m = np.zeros_like(params)
    v = np.zeros_like(params)
    losses = []
    s = 0
    for _ in range(epochs):
        for b in range(n_batches):
            sl = slice(b * batch, (b + 1) * batch)
            loss, g = loss_and_grads(params, x_all[sl], target[sl], emulate_bf16)
            params, m, v = adam_step(params, g, m, v, s, cosine_lr(lr0, s, total))
            losses.append(loss)
            s += 1
    return params, np.array(losses)


def infer(params, field32, X, family: int, I: int, m: int, audit_frac: float, tol_rel_rms: float,
          emulate_bf16: bool = False):
    """Learned interpolation with the audit and fallback; returns (u, audit_rms, fell_back)."""
    field32 = np.asarray(field32, dtype=np.float32)
    narrow = OI.interp_vec(field32, X, K.LAGRANGE, 4, 0)
    y, _ = forward(params, bf16_bits_to_f64(features(field32, X)), emulate_bf16)
    u = narrow + y
    k = max(1, int(round(1.0 / audit_frac)))
    idx = np.arange(0, X.shape[0], k)
    wide_a = OI.interp_vec(field32, X[idx], family, I, m)
    err = u[idx] - wide_a
    audit = float(np.sqrt(np.mean(err * err)) / np.sqrt(np.mean(wide_a * wide_a))) if idx.size else 0.0
    if audit > tol_rel_rms:
        return OI.interp_vec(field32, X, family, I, m), audit, True
    return u, audit, False


def linear_floor(feats_bits, target, n_fit: int):
    """Residual RMS of the best affine map from the 195 features to the target,
    fitted by least squares on the first n_fit pairs and evaluated on the rest:
    a reference point for what the network learns."""
    x = bf16_bits_to_f64(feats_bits)
    A = np.concatenate([x, np.ones((x.shape[0], 1))], axis=1)
    coef, *_ = np.linalg.lstsq(A[:n_fit], target[:n_fit], rcond=None)
    res = A[n_fit:] @ coef - target[n_fit:]
    return float(np.sqrt(np.mean(res * res)))
