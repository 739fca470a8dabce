"""FP64 CPU oracle of the learned surrogate (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  It shares no code with the GPU path.

The surrogate predicts the full-radius FBS subpixel disparity from a cheap
small-radius FBS run.  Everything here is written from that definition:

* features     per pixel, the 8 lowest aggregated costs of the cheap run in
               ascending order (ties to the lower disparity) divided by the
               cost cap, the 8 matching disparities as (d - d_min)/(D - 1),
               and the left intensity / 255: 17 channels.
* network      four 3x3 'same' (zero-padded) convolutions 17 -> 32 -> 32 -> 32
               -> 1 with ReLU after the first three; the output is a residual
               added to the cheap subpixel disparity.
* loss         mean absolute error against the label disparity.
* optimiser    Adam (Kingma and Ba) on float32 master weights.

BF16 rounding points follow the GPU kernels (weights, features and hidden
activations are BF16; sums are exact reals here, float32 on the GPU):
:func:`forward` rounds where the kernels store BF16 when ``bf16=True`` and is
a plain float64 network when ``bf16=False`` (used for finite differences).
Layouts are channel-last: activations [H][W][C]; weights [3][3][Cout][Cin]
with tap (ky, kx) at image offset (ky - 1, kx - 1).
"""
from __future__ import annotations

from typing import Dict, List, Tuple

import numpy as np

CH = (17, 32, 32, 32, 1)
K_TOP = 8


def bf16(x) -> np.ndarray:
    """Round to bfloat16 (round to nearest, ties to even), returned as float64."""
    a = np.asarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    nan = np.isnan(a)
    if nan.any():
        out[nan] = np.nan
    return out


def features(agg: np.ndarray, left: np.ndarray, d_min: int, tau: float) -> np.ndarray:
    """17-channel features [H][W][17] (float64, not rounded) from a [D][H][W] volume.

    Per pixel, the 8 lowest aggregated costs in exact ascending order (equal
    costs: the lower disparity first) divided by the cost cap, their
    disparity indices (d - d_min) / (D - 1) in the same order, and the left
    intensity / 255.  Costs are compared as given (float64 of the volume's
    values); nothing is truncated or re-encoded.
    """
    D, H, W = agg.shape
    a = np.asarray(agg, dtype=np.float64)
    order = np.argsort(a, axis=0, kind="stable")[:K_TOP]            # ascending, ties to lower d
    top = np.take_along_axis(a, order, axis=0)
    f = np.empty((H, W, 2 * K_TOP + 1))
    f[..., :K_TOP] = np.moveaxis(top / float(tau), 0, -1)
    denom = max(D - 1, 1)
    f[..., K_TOP:2 * K_TOP] = np.moveaxis(order.astype(np.float64) / denom, 0, -1)
    f[..., 2 * K_TOP] = left.astype(np.float64) / 255.0
    del d_min
    return f


def init_params(seed: int) -> Dict[str, np.ndarray]:
    """He-style initial weights (float32 masters), zero biases; last layer small."""
    rng = np.random.default_rng(seed)
    p = {}
    for l in range(4):
        cin, cout = CH[l], CH[l + 1]
        std = np.sqrt(2.0 / (9 * cin)) * (0.1 if l == 3 else 1.0)
        p[f"w{l}"] = rng.normal(0.0, std, size=(3, 3, cout, cin)).astype(np.float32)
        p[f"b{l}"] = np.zeros(cout, dtype=np.float32)
    return p


def conv3x3(x: np.ndarray, w: np.ndarray, b: np.ndarray) -> np.ndarray:
    """'same' 3x3 correlation: y[p, co] = sum_{ky,kx,ci} w[ky,kx,co,ci] x[p+(ky-1,kx-1), ci] + b."""
    H, W, _ = x.shape
    xp = np.pad(x, ((1, 1), (1, 1), (0, 0)))
    y = np.zeros((H, W, w.shape[2])) + b.astype(np.float64)
    for ky in range(3):
        for kx in range(3):
            y += xp[ky:ky + H, kx:kx + W, :] @ w[ky, kx].astype(np.float64).T
    return y


def forward(feat: np.ndarray, params: Dict[str, np.ndarray], bf16_points: bool = True):
    """Returns (residual [H][W], activations [a0..a3], pre-activations [z0..z2]).

    a0 is the (rounded) feature map; a_{l+1} = relu(z_l) rounded to BF16."""
    q = bf16 if bf16_points else (lambda v: np.asarray(v, dtype=np.float64))
    acts = [q(feat)]
    pres = []
    for l in range(4):
        z = conv3x3(acts[-1], q(params[f"w{l}"]), params[f"b{l}"])
        if l < 3:
            pres.append(z)
            acts.append(q(np.maximum(z, 0.0)))
        else:
            return z[..., 0], acts, pres
    raise AssertionError


def l1_loss_grad(pred: np.ndarray, label: np.ndarray) -> Tuple[float, np.ndarray]:
    """Mean |pred - label| and its gradient sign(pred - label) / N."""
    diff = pred - label
    return float(np.mean(np.abs(diff))), np.sign(diff) / diff.size


def backward(g_out: np.ndarray, acts: List[np.ndarray], params: Dict[str, np.ndarray],
             bf16_points: bool = True) -> Dict[str, np.ndarray]:
    """Gradients of all weights and biases given dL/d(residual) [H][W].

    With bf16_points the gradient flowing into each conv is rounded to BF16
    (as the kernels store it), and weights enter as their BF16 copies."""
    q = bf16 if bf16_points else (lambda v: np.asarray(v, dtype=np.float64))
    grads = {}
    g = g_out[..., None].astype(np.float64)                         # dL/dz3
    for l in (3, 2, 1, 0):
        x = acts[l]
        H, W, cin = x.shape
        xp = np.pad(x, ((1, 1), (1, 1), (0, 0)))
        gq = q(g)
        gw = np.zeros((3, 3, g.shape[2], cin))
        for ky in range(3):
            for kx in range(3):
                gw[ky, kx] = gq.reshape(-1, g.shape[2]).T @ xp[ky:ky + H, kx:kx + W, :].reshape(-1, cin)
        grads[f"w{l}"] = gw
        grads[f"b{l}"] = gq.reshape(-1, g.shape[2]).sum(axis=0)
        if l == 0:
            break
        # dL/dx: full convolution with the flipped kernel, then the ReLU mask
        wq = q(params[f"w{l}"]).astype(np.float64)
        gp = np.pad(gq, ((1, 1), (1, 1), (0, 0)))
        gx = np.zeros((H, W, cin))
        for ky in range(3):
            for kx in range(3):
                gx += gp[2 - ky:2 - ky + H, 2 - kx:2 - kx + W, :] @ wq[ky, kx]
        g = gx * (acts[l] > 0)
    return grads


def adam_step(params, grads, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (float64 arithmetic on float32 masters); returns new state."""
    t = state.get("t", 0) + 1
    new = {"t": t}
    out = {}
    for k, w in params.items():
        g = np.asarray(grads[k], dtype=np.float64)
        m = b1 * state.get("m_" + k, np.zeros_like(g)) + (1 - b1) * g
        v = b2 * state.get("v_" + k, np.zeros_like(g)) + (1 - b2) * g * g
        mh = m / (1 - b1 ** t)
        vh = v / (1 - b2 ** t)
        out[k] = (w.astype(np.float64) - lr * mh / (np.sqrt(vh) + eps)).astype(np.float32)
        new["m_" + k], new["v_" + k] = m, v
    return out, new
