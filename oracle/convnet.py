"""FP64 reference of the learned coarse propagator's network -- TEST INFRASTRUCTURE ONLY.

Complex arithmetic throughout (independent of the GPU kernels, which run the complex
layers as real convolutions on (re, im) channel pairs).  Network: 4 valid 5x5 complex
convolutions 1 -> C -> C -> C -> 1 with complex biases, CReLU (ReLU of the real and the
imaginary part) after layers 1-3.  Gradients use the Wirtinger pair convention
g = dL/dRe + i dL/dIm: for y = w x, g_w = g_y conj(x) and g_x = g_y conj(w).
Parameters are a list of (W[co][ci][5][5], b[co]) complex arrays.
"""
from __future__ import annotations

import numpy as np


def conv_valid(x: np.ndarray, w: np.ndarray, b: np.ndarray) -> np.ndarray:
    """x[B][ci][H][W], w[co][ci][5][5] -> y[B][co][H-4][W-4] = b + sum_ci sum_k w x(p+k)."""
    B, ci, H, W = x.shape
    co = w.shape[0]
    y = np.zeros((B, co, H - 4, W - 4), dtype=np.complex128) + b[None, :, None, None]
    for ky in range(5):
        for kx in range(5):
            patch = x[:, :, ky:ky + H - 4, kx:kx + W - 4]               # [B][ci][h][w]
            y += np.einsum("oc,bchw->bohw", w[:, :, ky, kx], patch)
    return y


def crelu(z: np.ndarray) -> np.ndarray:
    return np.maximum(z.real, 0.0) + 1j * np.maximum(z.imag, 0.0)


def forward(params, x: np.ndarray):
    """Returns the output and the list of layer inputs (for backward)."""
    acts = [x]
    h = x
    for l, (w, b) in enumerate(params):
        pre = conv_valid(h, w, b)
        h = crelu(pre) if l < 3 else pre
        acts.append(h)
    return h, acts


def rweights(row0: np.ndarray, H: int) -> np.ndarray:
    m = row0[:, None] + np.arange(H)[None, :]
    w = m.astype(np.float64)
    w[m == 0] = 0.125
    return w


def loss(out: np.ndarray, tgt: np.ndarray, row0: np.ndarray) -> float:
    w = rweights(row0, out.shape[2])[:, None, :, None]
    num = np.sum(w * np.abs(out - tgt) ** 2, axis=(1, 2, 3))
    den = np.sum(w * np.abs(tgt) ** 2, axis=(1, 2, 3))
    return float(np.mean(num / den))


def backward(params, acts, out, tgt, row0):
    """Wirtinger-pair gradients of loss(forward(params, x)) for each (W, b)."""
    B = out.shape[0]
    w = rweights(row0, out.shape[2])[:, None, :, None]
    den = np.sum(w * np.abs(tgt) ** 2, axis=(1, 2, 3))[:, None, None, None]
    g = 2.0 * w * (out - tgt) / (B * den)
    grads = [None] * 4
    for l in range(3, -1, -1):
        wgt, _ = params[l]
        x = acts[l]
        _, _, H, W = x.shape
        gw = np.zeros_like(wgt)
        gx = np.zeros_like(x)
        for ky in range(5):
            for kx in range(5):
                patch = x[:, :, ky:ky + H - 4, kx:kx + W - 4]
                gw[:, :, ky, kx] = np.einsum("bohw,bchw->oc", g, np.conj(patch))
                gx[:, :, ky:ky + H - 4, kx:kx + W - 4] += np.einsum("bohw,oc->bchw", g, np.conj(wgt[:, :, ky, kx]))
        gb = np.sum(g, axis=(0, 2, 3))
        grads[l] = (gw, gb)
        if l > 0:
            pre_sign = acts[l]  # post-activation of layer l-1; ReLU passes where it is > 0
            g = (gx.real * (pre_sign.real > 0)) + 1j * (gx.imag * (pre_sign.imag > 0))
    return grads


def flat(params) -> np.ndarray:
    """Same layout as the GPU parameter buffer: per layer W as (re, im) pairs, then b."""
    parts = []
    for w, b in params:
        parts.append(np.stack([w.real, w.imag], axis=-1).reshape(-1))
        parts.append(np.stack([b.real, b.imag], axis=-1).reshape(-1))
    return np.concatenate(parts)


def unflat(vec: np.ndarray, channels: int):
    cin = [1, channels, channels, channels]
    cout = [channels, channels, channels, 1]
    out, o = [], 0
    for ci, co in zip(cin, cout):
        nw = co * ci * 25
        w = vec[o:o + 2 * nw].reshape(co, ci, 5, 5, 2)
        o += 2 * nw
        b = vec[o:o + 2 * co].reshape(co, 2)
        o += 2 * co
        out.append((w[..., 0] + 1j * w[..., 1], b[:, 0] + 1j * b[:, 1]))
    return out
