"""Seeded synthetic inputs shared by the HIP path, its tests and the oracle tests.

This module only *draws* data: query points, cloth grids, network parameters,
meshes and training samples.  It holds none of the collision method's
arithmetic (no network evaluation, no gradients, no distances), so both sides
of every parity test can take their inputs from here without sharing any
computation.  Every generator uses numpy's PCG64 (``default_rng(seed)``),
draws in float64 and stores float32 where the value is a network input or a
parameter.

Parameter layout (flat float32, the concatenation of ``nn.Linear`` weight then
bias): for each hidden layer l = 1..L, W_l row-major ``[width_l][K_l]`` then
``b_l[width_l]``, where ``K_1 = 3`` and ``K_l = width_{l-1}`` plus 3 when l is
the skip layer (hidden features first, then x, y, z); then ``w_o[width_L]`` and
``b_o[1]``.  Sec. 3.1, Eq. 1 defines the map ``f: R^3 -> R``; widths, depth,
skip and softplus beta are build choices of the workloads below.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "NetSpec", "layer_shapes", "param_count", "init_geometric", "init_normal",
    "uniform_points", "cloth_grid", "icosphere", "displaced_icosphere",
    "surface_samples", "training_samples", "collider_set", "WORKLOADS",
]


@dataclass(frozen=True)
class NetSpec:
    """Shape of one collider network: L hidden layers of the given widths."""
    widths: tuple
    skip: int = 0          # 1-based hidden layer fed [h_{l-1}; x]; 0 = none
    beta: float = 100.0    # softplus sharpness
    fourier: int = 0       # m > 0: input gamma(x) = [sin 2 pi B x, cos 2 pi B x], B [m][3]

    @property
    def depth(self) -> int:
        return len(self.widths)


def layer_shapes(spec: NetSpec):
    """(out, in) of every affine map, hidden layers first, output layer last."""
    if spec.skip == 1 or spec.skip < 0 or spec.skip > spec.depth:
        raise ValueError("skip must be 0 or in [2, depth]")
    if spec.fourier and spec.skip:
        raise ValueError("a Fourier-feature net has no skip input")
    shapes = []
    prev = 2 * spec.fourier if spec.fourier else 3
    for l, w in enumerate(spec.widths, start=1):
        k = prev + (3 if l == spec.skip else 0)
        shapes.append((int(w), int(k)))
        prev = int(w)
    shapes.append((1, prev))
    return shapes


def param_count(spec: NetSpec) -> int:
    """Flat parameters: [B (m x 3, Fourier nets only)], then W_l, b_l, ..., w_o, b_o."""
    return 3 * spec.fourier + sum(o * i + o for o, i in layer_shapes(spec))


def init_fourier(spec: NetSpec, seed: int, sigma: float = 2.0) -> np.ndarray:
    """Fourier-feature net (Sec. 3.1, Fourier features): B ~ N(0, sigma^2) [m][3],
    hidden W ~ N(0, 1/K), biases N(0, 0.01^2), output w_o ~ N(0, 1/W)."""
    rng = np.random.default_rng(seed)
    parts = [rng.normal(0.0, sigma, size=3 * spec.fourier)]
    for o, i in layer_shapes(spec):
        parts.append(rng.normal(0.0, 1.0 / math.sqrt(i), size=o * i))
        parts.append(rng.normal(0.0, 0.01, size=o))
    return np.concatenate(parts).astype(np.float32)


def _pack(mats):
    return np.concatenate([m.ravel() for pair in mats for m in pair]).astype(np.float32)


def init_geometric(spec: NetSpec, seed: int, radius: float = 0.5) -> np.ndarray:
    """Geometric initialisation (Atzmon & Lipman, SAL) so that f(x) ~ |x| - radius.

    Hidden W ~ N(0, 2/width_out), b = 0; output w_o ~ N(sqrt(pi)/sqrt(width_L),
    1e-4^2), b_o = -radius.  The x-columns of the skip layer are zero so the
    construction still approximates the sphere.
    """
    rng = np.random.default_rng(seed)
    mats = []
    shapes = layer_shapes(spec)
    for l, (o, i) in enumerate(shapes[:-1], start=1):
        W = rng.normal(0.0, math.sqrt(2.0) / math.sqrt(o), size=(o, i))
        if l == spec.skip:
            W[:, i - 3:] = 0.0
        mats.append((W, np.zeros(o)))
    o, i = shapes[-1]
    wo = rng.normal(math.sqrt(math.pi) / math.sqrt(i), 1e-4, size=(1, i))
    mats.append((wo, np.array([-radius])))
    return _pack(mats)


def init_normal(spec: NetSpec, seed: int, std: float = 0.02) -> np.ndarray:
    """Every weight (output layer included) ~ N(0, std^2); every bias 0."""
    rng = np.random.default_rng(seed)
    mats = [(rng.normal(0.0, std, size=(o, i)), np.zeros(o)) for o, i in layer_shapes(spec)]
    return _pack(mats)


def uniform_points(n: int, seed: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=(n, 3)).astype(np.float32)


def _draw_wave_terms(rng):
    terms = []
    while len(terms) < 3:
        a, b = rng.integers(-2, 3, size=2)
        if a == 0 and b == 0:
            continue
        terms.append((float(a), float(b), float(rng.uniform(0.0, 2.0 * math.pi))))
    return terms


def cloth_grid(nx: int = 1000, ny: int = 1000, seed: int = 2, x0: float = -0.999,
               y0: float | None = None, spacing: float = 2e-3, amp: float = 0.1,
               jitter: float = 0.01) -> np.ndarray:
    """A rectangular cloth of nx*ny vertices draped over a smooth height field.

    Vertex (i, j) sits at x = x0 + spacing*i, y = y0 + spacing*j (index j*nx+i),
    z = amp * mean_k sin(2 pi (a_k x + b_k y) + phi_k) with three integer
    wave vectors a_k, b_k in {-2..2} (not both 0) and phases in [0, 2 pi);
    then every coordinate gets N(0, jitter^2) noise.  The paper's cloth is a
    rectangular quad grid (Sec. 4.1).
    """
    rng = np.random.default_rng(seed)
    terms = _draw_wave_terms(rng)
    y0 = x0 if y0 is None else y0
    xs = x0 + spacing * np.arange(nx, dtype=np.float64)
    ys = y0 + spacing * np.arange(ny, dtype=np.float64)
    X, Y = np.meshgrid(xs, ys)  # row j = y index
    Z = np.zeros_like(X)
    for a, b, ph in terms:
        Z += np.sin(2.0 * math.pi * (a * X + b * Y) + ph)
    Z *= amp / 3.0
    P = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    P += rng.normal(0.0, jitter, size=P.shape)
    return P.astype(np.float32)


def icosphere(level: int, radius: float = 1.0):
    """Vertices (float64 [V,3]) and outward-oriented faces (int32 [F,3])."""
    t = (1.0 + math.sqrt(5.0)) / 2.0
    V = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0),
         (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
         (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    F = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
         (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
         (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
         (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    verts = [np.array(v, dtype=np.float64) / np.linalg.norm(v) for v in V]
    faces = list(F)
    for _ in range(level):
        cache = {}

        def mid(a, b):
            key = (a, b) if a < b else (b, a)
            if key not in cache:
                m = verts[a] + verts[b]
                verts.append(m / np.linalg.norm(m))
                cache[key] = len(verts) - 1
            return cache[key]

        nf = []
        for a, b, c in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = nf
    Vn = np.asarray(verts) * radius
    Fn = np.asarray(faces, dtype=np.int32)
    # orient every face outward (star-shaped about the origin)
    a, b, c = Vn[Fn[:, 0]], Vn[Fn[:, 1]], Vn[Fn[:, 2]]
    flip = np.einsum("ij,ij->i", np.cross(b - a, c - a), a + b + c) < 0
    Fn[flip] = Fn[flip][:, [0, 2, 1]]
    return Vn, Fn


def displaced_icosphere(level: int = 6, seed: int = 3, radius: float = 0.5, amp: float = 0.05):
    """Watertight star-shaped mesh: icosphere with smooth radial displacement.

    r(u) = radius + amp * mean_k sin(omega_k (d_k . u) + phi_k), with random
    unit d_k, omega_k in {1,2,3}*pi and phi_k in [0, 2 pi).
    """
    rng = np.random.default_rng(seed)
    V, F = icosphere(level, 1.0)
    d = rng.normal(size=(3, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    om = math.pi * rng.integers(1, 4, size=3)
    ph = rng.uniform(0.0, 2.0 * math.pi, size=3)
    s = np.sin((V @ d.T) * om + ph).mean(axis=1)
    return V * (radius + amp * s)[:, None], F


def surface_samples(V, F, n: int, rng, sigma: float = 0.01):
    """Area-uniform points on the mesh plus isotropic N(0, sigma^2) offsets."""
    a, b, c = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]
    area = 0.5 * np.linalg.norm(np.cross(b - a, c - a), axis=1)
    tri = rng.choice(len(F), size=n, p=area / area.sum())
    u, v = rng.random(n), rng.random(n)
    fold = u + v > 1.0
    u[fold], v[fold] = 1.0 - u[fold], 1.0 - v[fold]
    P = a[tri] + u[:, None] * (b[tri] - a[tri]) + v[:, None] * (c[tri] - a[tri])
    return P + rng.normal(0.0, sigma, size=P.shape)


def training_samples(V, F, n: int, seed: int = 4, near_frac: float = 0.5):
    """Training points: near-surface and uniform in [-1,1]^3 (Sec. 3.1 sampling)."""
    rng = np.random.default_rng(seed)
    n_near = int(round(n * near_frac))
    near = surface_samples(V, F, n_near, rng)
    uni = rng.uniform(-1.0, 1.0, size=(n - n_near, 3))
    return np.concatenate([near, uni]).astype(np.float32)


def collider_set(seed: int = 5, n_nets: int = 16, total: int = 4_000_000,
                 lo: int = 10_000, hi: int = 1_000_000):
    """Several collider networks of uneven shape, each with its own cloth patch."""
    rng = np.random.default_rng(seed)
    widths = rng.choice([128, 256, 512], size=n_nets)
    depths = rng.integers(4, 9, size=n_nets)
    raw = np.exp(rng.uniform(math.log(lo), math.log(hi), size=n_nets))
    counts = np.clip(np.round(raw * total / raw.sum()), lo, hi).astype(np.int64)
    nets = []
    for i in range(n_nets):
        spec = NetSpec(widths=(int(widths[i]),) * int(depths[i]))
        side = int(math.ceil(math.sqrt(counts[i])))
        ny = int(math.ceil(counts[i] / side))
        step = 1.8 / max(side - 1, 1)
        pts = cloth_grid(side, ny, seed=1000 + i, x0=-0.9, y0=-0.9, spacing=step)[: counts[i]]
        nets.append({"spec": spec, "params": init_geometric(spec, 100 + i), "points": pts})
    return nets


@dataclass(frozen=True)
class Workload:
    name: str
    spec: NetSpec
    n: int
    eps: float = 0.005
    notes: str = ""
    extra: dict = field(default_factory=dict)


# The named workloads: small FP32 sphere check; cloth query at scale;
# fitting; FP8/BF16 precision; batched colliders.
WORKLOADS = {
    "sphere64": Workload("sphere64", NetSpec((64, 64, 64)), 4096,
                         notes="3->64x3->1, geometric init r=0.5 seed 0, uniform points seed 1"),
    "cloth1m": Workload("cloth1m", NetSpec((256,) * 8, skip=5), 1_000_000,
                        notes="3->256x8->1, skip into layer 5, N(0,0.02) seed 0, 1000x1000 cloth seed 2"),
    "fit_icosphere": Workload("fit_icosphere", NetSpec((256,) * 8, skip=5), 1_000_000,
                              notes="displaced icosphere level 6 seed 3, samples seed 4"),
    "wide4m": Workload("wide4m", NetSpec((512,) * 8, skip=5), 4_000_000,
                       notes="3->512x8->1, skip 5, geometric init seed 0, uniform seed 1"),
}


def workload_inputs(name: str, n: int | None = None, init: str | None = None):
    """(spec, params float32, points float32 [n,3], eps) for a named workload."""
    w = WORKLOADS[name]
    if name == "sphere64":
        params = init_geometric(w.spec, 0)
        pts = uniform_points(n or w.n, 1)
    elif name == "cloth1m":
        params = init_normal(w.spec, 0) if init in (None, "normal") else init_geometric(w.spec, 0)
        pts = cloth_grid(1000, 1000, seed=2)
        if n is not None:
            pts = pts[:n]
    elif name == "wide4m":
        params = init_geometric(w.spec, 0) if init in (None, "geometric") else init_normal(w.spec, 0)
        pts = uniform_points(n or w.n, 1)
    else:
        raise KeyError(name)
    return w.spec, params, np.ascontiguousarray(pts), w.eps
