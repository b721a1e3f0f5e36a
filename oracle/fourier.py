"""FP64 oracle of a Fourier-feature SDF network -- TEST INFRASTRUCTURE ONLY.

Sec. 3.1 names an MLP with Fourier features as its second architecture (the
mapping of Tancik et al.), and Sec. 4.3 times such nets: the input point x is
mapped to gamma(x) = [sin(2 pi B x), cos(2 pi B x)] (B an m x 3 matrix drawn
once and kept fixed) and gamma(x) feeds the softplus MLP of Eq. 1 in place of
x.  The input gradient (Sec. 3.2, back-propagation) continues through the
mapping: d gamma_j / dx = 2 pi cos(2 pi b_j.x) b_j for the sine half and
-2 pi sin(2 pi b_j.x) b_j for the cosine half.

Plain numpy in float64, one matrix product per layer; no blocking or fusion.
Flat parameters: B (m x 3, row-major), then W_l [w_l][K_l] and b_l for every
hidden layer (K_1 = 2m), then w_o and b_o.  No skip input.
"""
from __future__ import annotations

import numpy as np


def _layers(spec, P):
    m = spec.fourier
    off = 3 * m
    B = P[:off].reshape(m, 3)
    Ws, bs = [], []
    prev = 2 * m
    for w in spec.widths:
        Ws.append(P[off:off + w * prev].reshape(w, prev))
        off += w * prev
        bs.append(P[off:off + w])
        off += w
        prev = w
    wo, bo = P[off:off + prev], P[off + prev]
    if off + prev + 1 != P.size:
        raise ValueError("params has %d values, expected %d" % (P.size, off + prev + 1))
    return B, Ws, bs, wo, bo


def softplus(z, beta):
    return np.maximum(z, 0.0) + np.log1p(np.exp(-beta * np.abs(z))) / beta


def sigmoid(z, beta):
    a = beta * z
    e = np.exp(-np.abs(a))
    return np.where(a >= 0, 1.0 / (1.0 + e), e / (1.0 + e))


def mlp_eval(spec, params, pts, grad=True):
    """f (n,) and the input gradient (n, 3), float64."""
    P = np.asarray(params, dtype=np.float64).ravel()
    X = np.asarray(pts, dtype=np.float64).reshape(-1, 3)
    B, Ws, bs, wo, bo = _layers(spec, P)
    phase = 2.0 * np.pi * (X @ B.T)                      # (n, m)
    h = np.concatenate([np.sin(phase), np.cos(phase)], axis=1)
    zs = []
    for W, b in zip(Ws, bs):
        z = h @ W.T + b
        zs.append(z)
        h = softplus(z, spec.beta)
    f = h @ wo + bo
    if not grad:
        return f
    d = wo[None, :] * sigmoid(zs[-1], spec.beta)         # dLoss/dz_L with f as the loss
    for l in range(len(Ws) - 1, 0, -1):
        d = (d @ Ws[l]) * sigmoid(zs[l - 1], spec.beta)
    u = d @ Ws[0]                                        # d f / d gamma, (n, 2m)
    m = B.shape[0]
    gs = u[:, :m] * np.cos(phase) - u[:, m:] * np.sin(phase)   # d f / d (B x) / (2 pi)
    g = 2.0 * np.pi * (gs @ B)
    return f, g
