"""Numpy model of the operand roundings of the fused 16-bit / FP8 kernels.

Test infrastructure: it predicts how far a given operand scheme can land from
the FP64 result on a given network, without a GPU, so that tolerances of the
GPU tests and the choice of the headline precision rest on a committed
calculation.  It follows the structure of the collision path (Sec. 3.1, Eq. 1
forward; Sec. 3.2 reverse-mode input gradient) with every product of the
hidden contractions formed from rounded operands and summed exactly (FP64):
the FP32 accumulation of the matrix cores adds about 2^-24 sqrt(K) relative,
far below the operand roundings modelled here.

What is rounded, as in the kernels:
  * forward: the hidden weights W_l and the incoming activations r = kappa h
    (kappa = beta log2 e), both per the scheme's forward representation;
  * reverse: W_l^T and the back-propagated errors delta_l, per the scheme's
    reverse representation;
  * the sigmoids of the reverse sweep are recovered from the stored (rounded)
    r as 1 - 2^-r, the way the kernels avoid storing pre-activations;
  * layer 1 (K = 3), the skip x-columns, the output layer, biases and the
    normal stay FP32 (modelled as exact).

Representations of one operand:
  "bf16", "fp16"      one 16-bit value (round to nearest even);
  "bf16x2"            a BF16 pair hi + lo, lo = bf16(v - hi);
  "fp16x2"            an FP16 pair with the low part scaled by 2^11;
  "e4m3"              OCP E4M3 with a power-of-two scale per 32-element block
                      of K (largest scaled magnitude in (224, 448]);
  "exact"             no rounding.
A product scheme is a list of (A representation part, B representation part)
terms, e.g. BF16x3 = [(hi, hi), (hi, lo), (lo, hi)].
"""
from __future__ import annotations

import math

import numpy as np

KAPPA_PER_BETA = 1.0 / math.log(2.0)  # kappa = beta / ln 2


# ----------------------------------------------------------------- roundings

def round_bf16(x):
    """FP64 -> FP32 -> BF16 (round to nearest even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = ((u + 0x7FFF + lsb) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def round_fp16(x):
    return np.asarray(x, dtype=np.float32).astype(np.float16).astype(np.float64)


def round_e4m3(x):
    """OCP E4M3 ("fn": bias 7, no infinities, largest finite 448), round to
    nearest even, saturating; subnormals down to 2^-9."""
    x = np.asarray(x, dtype=np.float64)
    a = np.abs(x)
    _, e = np.frexp(a)  # a = m 2^e, m in [0.5, 1)
    step = np.ldexp(1.0, np.maximum(e - 4, -9))  # 3 fraction bits; subnormal step 2^-9
    q = np.round(a / step) * step  # numpy rounds half to even
    q = np.minimum(q, 448.0)
    return np.sign(x) * q


def split(x, fmt):
    """(hi, lo) parts of x in a 2-term representation (lo = 0 for 1 term)."""
    if fmt == "exact":
        return x, np.zeros_like(x)
    if fmt == "bf16":
        return round_bf16(x), np.zeros_like(x)
    if fmt == "fp16":
        return round_fp16(x), np.zeros_like(x)
    if fmt == "bf16x2":
        hi = round_bf16(x)
        return hi, round_bf16(x - hi)
    if fmt == "fp16x2":
        hi = round_fp16(x)
        return hi, round_fp16((x - hi) * 2048.0) / 2048.0
    if fmt == "fp16m1":  # FP16 of (x - 1), for values near 1 (activations at z = 0)
        return round_fp16(x - 1.0) + 1.0, np.zeros_like(x)
    if fmt == "bf16m1":
        return round_bf16(x - 1.0) + 1.0, np.zeros_like(x)
    if fmt == "e4m3_t":  # weights: one power-of-two scale per layer from the largest weight
        return tensorscaled_e4m3(x), np.zeros_like(x)
    if fmt == "e4m3_r4":  # forward activations enter as r / 4
        return round_e4m3(np.asarray(x) / 4.0) * 4.0, np.zeros_like(x)
    if fmt == "e4m3_rms":  # back-propagated errors with a power-of-two scale ~ 1/rms
        x = np.asarray(x, dtype=np.float64)
        rms = math.sqrt(float(np.mean(x * x))) + 1e-300
        sc = math.ldexp(1.0, int(round(-math.log2(rms))))
        return round_e4m3(x * sc) / sc, np.zeros_like(x)
    raise ValueError(fmt)


def tensorscaled_e4m3(x):
    """E4M3 with one power-of-two scale for the whole tensor (largest scaled
    magnitude in (224, 448])."""
    x = np.asarray(x, dtype=np.float64)
    amax = np.abs(x).max()
    if amax == 0:
        return x
    s = math.ldexp(1.0, int(math.ceil(math.log2(amax / 448.0))))
    return round_e4m3(x / s) * s


def blockscaled_e4m3(x, axis, block=32):
    """E4M3 with one power-of-two scale per `block` consecutive elements along
    `axis` (the K axis of the contraction), chosen so the block's largest
    magnitude lands in (224, 448]."""
    x = np.moveaxis(np.asarray(x, dtype=np.float64), axis, -1)
    K = x.shape[-1]
    pad = (-K) % block
    xp = np.concatenate([x, np.zeros(x.shape[:-1] + (pad,))], axis=-1) if pad else x
    xb = xp.reshape(xp.shape[:-1] + (-1, block))
    amax = np.abs(xb).max(axis=-1, keepdims=True)
    with np.errstate(divide="ignore"):
        k = np.where(amax > 0, np.ceil(np.log2(np.where(amax > 0, amax, 1.0) / 448.0)), 0.0)
    s = np.ldexp(1.0, k.astype(np.int64))
    q = (round_e4m3(xb / s) * s).reshape(xp.shape)[..., :K]
    return np.moveaxis(q, -1, axis)


# --------------------------------------------------------------- the schemes

class Scheme:
    """How one contraction Y = A X (A: weights [M][K], X: operand [K][n]) is
    formed.  `terms` lists (part of A, part of X) products; parts are "hi",
    "lo" of the representations `a_fmt` / `x_fmt`, or "c" for the
    block-scaled E4M3 correction term sum_k (A-lo X-hi + A-hi X-lo)."""

    def __init__(self, name, a_fmt, x_fmt, terms, mfma_cost, stack=None):
        self.name, self.a_fmt, self.x_fmt, self.terms, self.cost = name, a_fmt, x_fmt, terms, mfma_cost
        # representation of the activations kept for the reverse sweep's sigmoids
        self.stack = stack or x_fmt

    def stored(self, r):
        hi, lo = split(r, self.stack)
        return hi + lo

    def contract(self, A, X):
        Ah, Al = split(A, self.a_fmt)
        Xh, Xl = split(X, self.x_fmt)
        parts = {"hi": (Ah, Xh), "lo": (Al, Xl)}
        Y = np.zeros((A.shape[0], X.shape[1]))
        for ta, tx in self.terms:
            if ta == "c":  # the two cross terms from block-scaled E4M3 operands (one K = 2K pass)
                Y += blockscaled_e4m3(A - Ah, 1) @ blockscaled_e4m3(Xh, 0)
                Y += blockscaled_e4m3(Ah, 1) @ blockscaled_e4m3(X - Xh, 0)
                continue
            if ta == "t":  # the same with one scale per operand tensor
                Y += tensorscaled_e4m3(A - Ah) @ tensorscaled_e4m3(Xh)
                Y += tensorscaled_e4m3(Ah) @ tensorscaled_e4m3(X - Xh)
                continue
            Y += parts[ta][0] @ parts[tx][1]
        return Y


def _plain(fmt, cost=1.0):
    return Scheme(fmt, fmt, fmt, [("hi", "hi")], cost)


SCHEMES = {
    "exact": _plain("exact", 0.0),
    "bf16": _plain("bf16"),
    "fp16": _plain("fp16"),
    # three BF16 products: hi*hi + hi*lo + lo*hi (the kernel's SDF_BF16X3)
    "bf16x3": Scheme("bf16x3", "bf16x2", "bf16x2", [("hi", "hi"), ("hi", "lo"), ("lo", "hi")], 3.0),
    # two products: only one operand carried as a pair
    "bf16_w2": Scheme("bf16_w2", "bf16x2", "bf16", [("hi", "hi"), ("lo", "hi")], 2.0),
    "bf16_x2": Scheme("bf16_x2", "bf16", "bf16x2", [("hi", "hi"), ("hi", "lo")], 2.0),
    "fp16_w2": Scheme("fp16_w2", "fp16x2", "fp16", [("hi", "hi"), ("lo", "hi")], 2.0),
    "fp16_x2": Scheme("fp16_x2", "fp16", "fp16x2", [("hi", "hi"), ("hi", "lo")], 2.0),
    # FP16 main product plus both cross terms on the FP8 matrix cores (K doubled
    # at twice the rate: the cost of one more 16-bit product)
    "fp16_c8": Scheme("fp16_c8", "fp16", "fp16", [("hi", "hi"), ("c", "c")], 2.0),
    "bf16_c8": Scheme("bf16_c8", "bf16", "bf16", [("hi", "hi"), ("c", "c")], 2.0),
    # the same with the reverse sweep's activations kept as a pair
    "fp16_c8p": Scheme("fp16_c8p", "fp16", "fp16", [("hi", "hi"), ("c", "c")], 2.0, stack="fp16x2"),
    "fp16p": Scheme("fp16p", "fp16", "fp16", [("hi", "hi")], 1.0, stack="fp16x2"),
    "bf16p": Scheme("bf16p", "bf16", "bf16", [("hi", "hi")], 1.0, stack="bf16x2"),
    "fp16m1": Scheme("fp16m1", "fp16", "fp16", [("hi", "hi")], 1.0, stack="fp16m1"),
    "fp16_t8": Scheme("fp16_t8", "fp16", "fp16", [("hi", "hi"), ("t", "t")], 2.0),
    "fp16_t8m1": Scheme("fp16_t8m1", "fp16", "fp16", [("hi", "hi"), ("t", "t")], 2.0, stack="fp16m1"),
    "fp16_c8m1": Scheme("fp16_c8m1", "fp16", "fp16", [("hi", "hi"), ("c", "c")], 2.0, stack="fp16m1"),
    # the kernel's SDF_FP8: E4M3 on both sides of every hidden contraction,
    # BF16 activations kept for the reverse sweep
    # BF16x3 contractions with a single 16-bit copy of the activations kept for the reverse sweep
    "bf16x3_s16": Scheme("bf16x3_s16", "bf16x2", "bf16x2", [("hi", "hi"), ("hi", "lo"), ("lo", "hi")], 3.0,
                         stack="fp16m1"),
    "bf16x3_sb": Scheme("bf16x3_sb", "bf16x2", "bf16x2", [("hi", "hi"), ("hi", "lo"), ("lo", "hi")], 3.0,
                        stack="bf16"),
    "fp8": Scheme("fp8", "e4m3_t", "e4m3_r4", [("hi", "hi")], 0.5, stack="bf16"),
    "fp8r": Scheme("fp8r", "e4m3_t", "e4m3_rms", [("hi", "hi")], 0.5),
}


# ------------------------------------------------------------------- network

def unpack(spec, params):
    """[(W_l, b_l)] for the hidden layers and (w_o, b_o), float64."""
    P = np.asarray(params, dtype=np.float64)
    o = 0
    layers = []
    prev = 3
    for l, w in enumerate(spec.widths, start=1):
        k = prev + (3 if l == spec.skip else 0)
        W = P[o:o + w * k].reshape(w, k)
        o += w * k
        b = P[o:o + w]
        o += w
        layers.append((W, b))
        prev = w
    wo = P[o:o + prev]
    bo = P[o + prev]
    assert o + prev + 1 == P.size, "parameter count"
    return layers, wo, bo


def emulate(spec, params, pts, fwd="exact", rev=None, sigma_from_stored=True):
    """f [n] and grad f [n][3] with the forward contractions formed by scheme
    `fwd` and the reverse ones by `rev` (default: the same)."""
    F, R = SCHEMES[fwd], SCHEMES[rev or fwd]
    layers, wo, bo = unpack(spec, params)
    kappa = spec.beta * KAPPA_PER_BETA
    X = np.asarray(pts, dtype=np.float64).T  # [3][n]
    L = len(layers)
    sig = []
    r = None
    for l, (W, b) in enumerate(layers, start=1):
        if l == 1:
            y = kappa * (W @ X + b[:, None])
        else:
            Wh = W[:, :W.shape[1] - (3 if l == spec.skip else 0)]
            y = F.contract(Wh, r) + kappa * b[:, None]
            if l == spec.skip:
                y += kappa * (W[:, -3:] @ X)
        # softplus and sigmoid in base-2 units: r = log2(1 + 2^y)
        r = np.maximum(y, 0.0) + np.log2(1.0 + np.exp2(-np.abs(y)))
        s_exact = 1.0 / (1.0 + np.exp2(-y))
        # the next contraction rounds r itself (F.contract); the reverse sweep
        # recovers sigma from r as kept on chip
        if F.name == "exact" or not sigma_from_stored or l == L:
            sig.append(s_exact)
        else:
            sig.append(1.0 - np.exp2(-F.stored(r)))
    f = (wo @ r) / kappa + bo
    # reverse sweep: delta_L = w_o * sigma_L, g = W_l^T delta_l, delta_{l-1} = g * sigma_{l-1}
    d = wo[:, None] * sig[-1]
    gx = np.zeros_like(X)
    for l in range(L, 0, -1):
        W = layers[l - 1][0]
        if l == 1:
            gx += W.T @ d
            break
        kh = W.shape[1] - (3 if l == spec.skip else 0)
        if l == spec.skip:
            gx += W[:, kh:].T @ d
        g = R.contract(W[:, :kh].T, d)
        d = g * sig[l - 2]
    return f, gx.T


def errors(f, g, f64, g64):
    """SDF error and normal-angle error (rad) statistics against FP64."""
    ferr = np.abs(f - f64)
    cr = np.linalg.norm(np.cross(g, g64), axis=1)
    ang = np.arctan2(cr, np.einsum("ij,ij->i", g, g64))
    return {"sdf_max": float(ferr.max()), "sdf_p99": float(np.quantile(ferr, 0.99)),
            "angle_max": float(ang.max()), "angle_p99": float(np.quantile(ang, 0.99))}


def scheme_errors(spec, params, pts, fwd, rev=None, ref=None):
    """errors() of a scheme against the exact model (or `ref` = (f64, g64))."""
    f64, g64 = ref if ref is not None else emulate(spec, params, pts, "exact")
    f, g = emulate(spec, params, pts, fwd, rev)
    return errors(f, g, f64, g64)
