"""FP64 reference of the warm-start network (test infrastructure).

The network maps the per-element field of an oversampled box to coefficients
of the starting block of the local eigensolver (a learned warm start; not in
the paper).  The structure follows the layer list this project fixes for it:
four 3x3x3 convolutions with zero padding 1 and strides 1, 1, 2, 2, each
followed by ReLU, a global average over the grid, and one affine map to
n_out values.

Layouts (all float64 NumPy):
  x      [B, C_in, D, D, D]
  conv w [C_out, C_in, 3, 3, 3], b [C_out]
  lin  w [n_out, C_last], b [n_out]
Output size of a stride-s convolution with padding 1: (D - 1) // s + 1.

BF16 storage (``bf16=True``): the input, the convolution weights and every
stored activation are rounded to bfloat16 (8 significant bits, round to
nearest, ties to even) and the sums are exact (FP64); biases, the pooled
vector and the affine map stay unrounded.  The gradient is the one of that
rounded network with respect to the unrounded parameters (the rounding is
passed straight through).

Only tests/, __graft_entry__.smoke() and bench.py's CPU baseline use this
module; the library never calls it.
"""
from __future__ import annotations

from typing import Dict, List, Sequence, Tuple

import numpy as np

STRIDES = (1, 1, 2, 2)


def out_size(d: int, stride: int) -> int:
    return (d - 1) // stride + 1


def bf16(x: np.ndarray) -> np.ndarray:
    """Round to the nearest bfloat16 value (ties to even), as float64.
    x = m 2^e with 0.5 <= |m| < 1; bfloat16 keeps 8 significant bits of m."""
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)
    return np.ldexp(np.rint(m * 256.0) / 256.0, e)


def conv3d(x: np.ndarray, w: np.ndarray, b: np.ndarray, stride: int) -> np.ndarray:
    """Cross-correlation with zero padding 1: y[n,o,i,j,k] = b[o] +
    sum_{c,p,q,r} w[o,c,p,q,r] x[n,c, s*i+p-1, s*j+q-1, s*k+r-1]."""
    n, c, d = x.shape[0], x.shape[1], x.shape[2]
    od = out_size(d, stride)
    xp = np.zeros((n, c, d + 2, d + 2, d + 2))
    xp[:, :, 1:-1, 1:-1, 1:-1] = x
    y = np.zeros((n, w.shape[0], od, od, od))
    y += b[None, :, None, None, None]
    lim = stride * (od - 1) + 1
    for p in range(3):
        for q in range(3):
            for r in range(3):
                patch = xp[:, :, p:p + lim:stride, q:q + lim:stride, r:r + lim:stride]
                y += np.einsum("oc,ncijk->noijk", w[:, :, p, q, r], patch)
    return y


def conv3d_backward(x: np.ndarray, w: np.ndarray, gy: np.ndarray, stride: int
                    ) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Gradients (gx, gw, gb) of conv3d for the output gradient gy."""
    n, c, d = x.shape[0], x.shape[1], x.shape[2]
    od = gy.shape[2]
    xp = np.zeros((n, c, d + 2, d + 2, d + 2))
    xp[:, :, 1:-1, 1:-1, 1:-1] = x
    gxp = np.zeros_like(xp)
    gw = np.zeros_like(w)
    lim = stride * (od - 1) + 1
    for p in range(3):
        for q in range(3):
            for r in range(3):
                sl = (slice(None), slice(None), slice(p, p + lim, stride), slice(q, q + lim, stride),
                      slice(r, r + lim, stride))
                gw[:, :, p, q, r] = np.einsum("noijk,ncijk->oc", gy, xp[sl])
                gxp[sl] += np.einsum("oc,noijk->ncijk", w[:, :, p, q, r], gy)
    gb = gy.sum(axis=(0, 2, 3, 4))
    return gxp[:, :, 1:-1, 1:-1, 1:-1], gw, gb


def init_params(c_in: int, width: int, n_out: int, seed: int) -> Dict[str, np.ndarray]:
    """He-style random initialisation (the GPU path is given the same values)."""
    rng = np.random.default_rng(seed)
    p: Dict[str, np.ndarray] = {}
    cin = c_in
    for l in range(4):
        fan = cin * 27
        p[f"w{l}"] = rng.standard_normal((width, cin, 3, 3, 3)) * np.sqrt(2.0 / fan)
        p[f"b{l}"] = np.zeros(width)
        cin = width
    p["wl"] = rng.standard_normal((n_out, width)) * np.sqrt(1.0 / width)
    p["bl"] = np.zeros(n_out)
    return p


def _stored(p: Dict[str, np.ndarray], use_bf16: bool) -> Dict[str, np.ndarray]:
    if not use_bf16:
        return p
    return {k: (bf16(v) if k in ("w0", "w1", "w2", "w3") else v) for k, v in p.items()}


def forward(p: Dict[str, np.ndarray], x: np.ndarray, use_bf16: bool = False
            ) -> Tuple[np.ndarray, List[np.ndarray]]:
    """Network output [B, n_out] and the activations needed by backward."""
    q = _stored(p, use_bf16)
    rnd = bf16 if use_bf16 else (lambda a: a)
    h = rnd(x)
    acts = [h]
    for l, s in enumerate(STRIDES):
        h = rnd(np.maximum(conv3d(h, q[f"w{l}"], q[f"b{l}"], s), 0.0))
        acts.append(h)
    g = h.mean(axis=(2, 3, 4))
    acts.append(g)
    return g @ p["wl"].T + p["bl"], acts


def backward(p: Dict[str, np.ndarray], acts: Sequence[np.ndarray], gout: np.ndarray,
             use_bf16: bool = False) -> Dict[str, np.ndarray]:
    """Gradients of sum(gout * forward(p, x)) with respect to every parameter."""
    p = _stored(p, use_bf16)
    grads: Dict[str, np.ndarray] = {}
    g = acts[-1]
    grads["wl"] = gout.T @ g
    grads["bl"] = gout.sum(axis=0)
    gg = gout @ p["wl"]                                    # [B, width]
    h = acts[4]
    vol = h.shape[2] * h.shape[3] * h.shape[4]
    gh = np.broadcast_to(gg[:, :, None, None, None] / vol, h.shape).copy()
    for l in range(3, -1, -1):
        gh = gh * (acts[l + 1] > 0.0)                      # ReLU
        gx, gw, gb = conv3d_backward(acts[l], p[f"w{l}"], gh, STRIDES[l])
        grads[f"w{l}"] = gw
        grads[f"b{l}"] = gb
        gh = gx
    return grads


def projector_loss(c: np.ndarray, c_star: np.ndarray) -> Tuple[float, np.ndarray]:
    """Subspace loss of predicted coefficients c [B, n, m] against label
    coefficients c_star [B, n, m] with orthonormal columns:
    L = sum_b |c_b c_b^T - P_b|_F^2, P_b = c*_b c*_b^T; returns (L, dL/dc).
    It is invariant under c_b -> c_b Q for orthogonal Q (only the spanned
    subspace of a prediction with orthonormal columns matters)."""
    loss = 0.0
    grad = np.zeros_like(c)
    for b in range(c.shape[0]):
        e = c[b] @ c[b].T - c_star[b] @ c_star[b].T
        loss += float(np.sum(e * e))
        grad[b] = 4.0 * e @ c[b]
    return loss, grad
