"""Pins of the FP64 oracle against facts the paper and the mathematics fix.

None of these compare the oracle with itself: each uses an independent
library routine (torch autograd), a closed form, an invariant, a second
algorithm, a hand-derived golden value or brute force.  CPU only.
"""
import json
import math
import os

import numpy as np
import pytest
import torch

import oracle
from paper_2110_01614_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- helpers

def torch_mlp(spec, params, pts):
    """f and grad f with torch float64 autograd, built independently from the flat layout."""
    P = torch.tensor(np.asarray(params, dtype=np.float64))
    x = torch.tensor(np.asarray(pts, dtype=np.float64), requires_grad=True)
    off, h = 0, x
    shapes = I.layer_shapes(spec)
    for l, (o, i) in enumerate(shapes[:-1], start=1):
        W = P[off:off + o * i].view(o, i)
        off += o * i
        b = P[off:off + o]
        off += o
        u = torch.cat([h, x], dim=1) if l == spec.skip else h
        # threshold 30: torch's linear branch differs from softplus by < exp(-30)/beta
        h = torch.nn.functional.softplus(u @ W.T + b, beta=spec.beta, threshold=30.0)
    _, i = shapes[-1]
    wo, bo = P[off:off + i], P[off + i]
    f = h @ wo + bo
    (g,) = torch.autograd.grad(f.sum(), x)
    return f.detach().numpy(), g.numpy()


def random_net(seed, widths, skip, scale=0.5):
    spec = I.NetSpec(tuple(widths), skip=skip, beta=100.0)
    rng = np.random.default_rng(seed)
    shapes = I.layer_shapes(spec)
    parts = []
    for o, i in shapes:
        parts.append(rng.normal(0, scale / math.sqrt(i), size=o * i))
        parts.append(rng.normal(0, 0.05, size=o))
    return spec, np.concatenate(parts).astype(np.float32)


NETS = [
    ((16, 16, 16), 0),
    ((24, 24, 24, 24, 24), 3),
    ((32,) * 8, 5),
    ((7, 11, 5), 2),
]


# ------------------------------------------------------- forward / gradient

@pytest.mark.parametrize("widths,skip", NETS)
def test_forward_and_gradient_match_torch_autograd(widths, skip):
    spec, params = random_net(1, widths, skip)
    x = I.uniform_points(300, 2)
    f, g = oracle.mlp_eval(spec, params, x)
    ft, gt = torch_mlp(spec, params, x)
    assert np.max(np.abs(f - ft)) <= 1e-12 * (1 + np.max(np.abs(ft)))
    assert np.max(np.abs(g - gt)) <= 1e-11 * (1 + np.max(np.abs(gt)))


@pytest.mark.parametrize("widths,skip", NETS)
def test_reverse_mode_equals_forward_mode(widths, skip):
    spec, params = random_net(3, widths, skip)
    x = I.uniform_points(200, 4)
    f1, g1 = oracle.mlp_eval(spec, params, x, mode="reverse")
    f2, g2 = oracle.mlp_eval(spec, params, x, mode="forward")
    assert np.array_equal(f1, f2)
    assert np.max(np.abs(g1 - g2)) <= 1e-12 * (1 + np.max(np.abs(g1)))


def test_gradient_matches_central_differences():
    spec = I.NetSpec((64, 64, 64))
    params = I.init_geometric(spec, 0)
    x = I.uniform_points(256, 1).astype(np.float64)
    _, g = oracle.mlp_eval(spec, params, x)
    h = 1e-6
    fd = np.empty_like(g)
    for c in range(3):
        e = np.zeros(3)
        e[c] = h
        fd[:, c] = (oracle.mlp_eval(spec, params, x + e, grad=False)
                    - oracle.mlp_eval(spec, params, x - e, grad=False)) / (2 * h)
    assert np.max(np.abs(fd - g)) < 1e-8


def plane_net(n, d, widths=(32, 32, 32, 32, 32, 32), skip=4, C=2.5, seed=5):
    """An MLP whose unit 0 carries n.x - d + C through every layer exactly.

    In softplus's linear regime (beta*z > 40, so exp(-beta z) < 1e-17 relative)
    every layer passes unit 0 on unchanged; the output reads only unit 0, so
    f(x) = n.x - d exactly and grad f = n.
    """
    spec = I.NetSpec(tuple(widths), skip=skip)
    rng = np.random.default_rng(seed)
    parts = []
    for l, (o, i) in enumerate(I.layer_shapes(spec)[:-1], start=1):
        W = rng.normal(0, 0.3, size=(o, i))
        b = rng.normal(0, 0.1, size=o)
        W[0, :] = 0.0
        if l == 1:
            W[0, :3] = n
            b[0] = C - d
        else:
            W[0, 0] = 1.0
            b[0] = 0.0
        parts += [W.ravel(), b]
    o, i = I.layer_shapes(spec)[-1]
    wo = np.zeros(i)
    wo[0] = 1.0
    parts += [wo, np.array([-C])]
    return spec, np.concatenate(parts)


def test_plane_embedded_in_mlp_is_exact():
    n = np.array([0.6, -0.48, 0.64])  # unit, exactly representable products
    d = 0.25
    spec, P = plane_net(n, d)
    x = I.uniform_points(500, 7).astype(np.float64)
    # pass FP64 params straight through (no float32 rounding of the construction)
    f, g = oracle.mlp_eval(spec, P, x)
    exact = x @ n - d
    assert np.max(np.abs(f - exact)) < 1e-14
    assert np.max(np.abs(g - n)) < 1e-15


def rotation(seed):
    """A proper rotation from a seeded unit quaternion."""
    q = np.random.default_rng(seed).normal(size=4)
    w, x, y, z = q / np.linalg.norm(q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                     [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                     [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def test_rigid_frame_moves_the_plane_in_closed_form():
    """Sec. 4.2: a collider moved by T = [R t; 0 1] is the plane n.x = d moved by
    T: f(p) = (R n).(p - t) - d, normal R n, and every hit lands on f = eps."""
    n = np.array([0.6, -0.48, 0.64])
    d, eps = 0.25, 0.01
    spec, P = plane_net(n, d)
    R, t = rotation(3), np.array([0.3, -0.2, 0.15])
    T = np.eye(4)
    T[:3, :3], T[:3, 3] = R, t
    x = I.uniform_points(800, 13).astype(np.float64)
    res = oracle.collide_project_rigid(spec, P, x, eps, T)
    Rn = R @ n
    assert np.max(np.abs(res["sdf"] - ((x - t) @ Rn - d))) < 1e-13
    assert np.max(np.abs(res["normal"] - Rn)) < 1e-13
    hit = res["hit"] == 1
    assert hit.any() and (~hit).any()
    assert np.max(np.abs((res["pts"][hit] - t) @ Rn - d - eps)) < 1e-13
    assert np.array_equal(res["pts"][~hit], x[~hit])


def test_rigid_frame_gradient_matches_differences_for_a_general_affine_map():
    """The gradient of p -> f(A^{-1}(p - t)) against central differences, with a
    non-orthogonal A (the transformation rule itself, not only rotations)."""
    spec, P = random_net(21, (16, 16, 16), 0)
    A = np.array([[1.2, 0.3, -0.1], [0.0, 0.9, 0.4], [0.2, -0.3, 1.1]])
    T = np.eye(4)
    T[:3, :3], T[:3, 3] = A, [0.1, 0.2, -0.3]
    x = I.uniform_points(50, 14).astype(np.float64)
    res = oracle.collide_project_rigid(spec, P, x, 0.0, T)
    h = 1e-6
    for c in range(3):
        e = np.zeros(3)
        e[c] = h
        fp = oracle.collide_project_rigid(spec, P, x + e, 0.0, T)["sdf"]
        fm = oracle.collide_project_rigid(spec, P, x - e, 0.0, T)["sdf"]
        assert np.max(np.abs((fp - fm) / (2 * h) - res["grad"][:, c])) < 1e-6


def torch_fourier_mlp(spec, params, pts):
    """Fourier-feature net with torch float64 autograd, from the flat layout."""
    P = torch.tensor(np.asarray(params, dtype=np.float64))
    x = torch.tensor(np.asarray(pts, dtype=np.float64), requires_grad=True)
    m = spec.fourier
    B = P[:3 * m].view(m, 3)
    off = 3 * m
    proj = 2 * math.pi * x @ B.T
    h = torch.cat([torch.sin(proj), torch.cos(proj)], dim=1)
    for o, i in I.layer_shapes(spec)[:-1]:
        W = P[off:off + o * i].view(o, i)
        off += o * i
        b = P[off:off + o]
        off += o
        h = torch.nn.functional.softplus(h @ W.T + b, beta=spec.beta, threshold=30.0)
    _, i = I.layer_shapes(spec)[-1]
    f = h @ P[off:off + i] + P[off + i]
    (g,) = torch.autograd.grad(f.sum(), x)
    return f.detach().numpy(), g.numpy()


@pytest.mark.parametrize("widths,m,sigma", [((32, 32), 16, 1.0), ((64,) * 4, 32, 3.0), ((24, 40, 16), 5, 2.0)])
def test_fourier_features_match_torch_autograd(widths, m, sigma):
    """Sec. 3.1 / 4.3 Fourier-feature input: f and grad f against torch autograd."""
    spec = I.NetSpec(tuple(widths), fourier=m)
    P = I.init_fourier(spec, 9, sigma)
    x = I.uniform_points(300, 16).astype(np.float64)
    f, g = oracle.mlp_eval(spec, P, x)
    ft, gt = torch_fourier_mlp(spec, P, x)
    assert np.max(np.abs(f - ft)) < 1e-12 * (1 + np.abs(ft).max())
    assert np.max(np.abs(g - gt)) < 1e-11 * (1 + np.abs(gt).max())


def test_fourier_gradient_matches_central_differences():
    spec = I.NetSpec((32, 32, 32), fourier=16)
    P = I.init_fourier(spec, 10, 2.0)
    x = I.uniform_points(40, 17).astype(np.float64)
    _, g = oracle.mlp_eval(spec, P, x)
    h = 1e-6
    for c in range(3):
        e = np.zeros(3)
        e[c] = h
        fd = (oracle.mlp_eval(spec, P, x + e, grad=False) - oracle.mlp_eval(spec, P, x - e, grad=False)) / (2 * h)
        assert np.max(np.abs(fd - g[:, c])) < 1e-6 * (1 + np.abs(g).max())


# ---------------------------------------------------------- collision step

def test_projection_onto_analytic_sphere_is_closed_form():
    r, eps = 0.5, 0.005
    x = I.uniform_points(4000, 11).astype(np.float64)
    x = x[np.linalg.norm(x, axis=1) > 1e-3]
    nx = np.linalg.norm(x, axis=1)
    f = nx - r
    g = x / nx[:, None]
    out, N, hit = oracle.collide(x, f, g, eps)
    assert np.array_equal(hit.astype(bool), f < eps)
    want = (r + eps) * x / nx[:, None]
    assert np.max(np.abs(out[hit == 1] - want[hit == 1])) < 1e-14
    assert np.array_equal(out[hit == 0], x[hit == 0])  # bit-identical non-hits
    assert np.max(np.abs(np.linalg.norm(N, axis=1) - 1)) < 1e-15


def test_projection_onto_plane_is_closed_form_and_idempotent():
    n = np.array([0.0, 0.6, 0.8])
    d, eps = 0.1, 0.01
    x = I.uniform_points(3000, 12).astype(np.float64)
    f = x @ n - d
    g = np.broadcast_to(n, x.shape)
    out, _, hit = oracle.collide(x, f, g, eps)
    want = x + ((eps - f) * (f < eps))[:, None] * n
    assert np.max(np.abs(out - want)) < 1e-15
    # a moved vertex sits at distance eps; not strictly below, so no second hit
    f2 = out @ n - d
    assert np.all(f2[hit == 1] >= eps - 1e-15)


def test_projection_policy_nan_and_zero_gradient():
    x = np.array([[0.1, 0.2, 0.3], [0.4, 0.5, 0.6], [-0.1, 0.0, 0.2]])
    f = np.array([np.nan, -0.2, 0.005])
    g = np.array([[1.0, 0.0, 0.0], [0.0, 0.0, 0.0], [0.0, 1.0, 0.0]])
    out, N, hit = oracle.collide(x, f, g, 0.005)
    assert list(hit) == [0, 1, 0]        # NaN < eps is false; f == eps is not a hit
    assert np.array_equal(out, x)         # zero gradient: N = 0, vertex not moved
    assert np.array_equal(N[1], [0.0, 0.0, 0.0])


def test_geometric_init_approximates_the_sphere():
    """The small sphere workload: 3->64x3->1, geometric init r=0.5, 4096 uniform points."""
    spec, params, x, _ = I.workload_inputs("sphere64")
    f, g = oracle.mlp_eval(spec, params, x)
    r = np.linalg.norm(x.astype(np.float64), axis=1)
    far = np.abs(r - 0.5) > 0.2
    assert np.all(np.sign(f[far]) == np.sign(r[far] - 0.5))
    sel = r > 0.1
    cosang = np.einsum("ij,ij->i", g[sel], x[sel]) / (np.linalg.norm(g[sel], axis=1) * r[sel])
    assert np.max(np.arccos(np.clip(cosang, -1, 1))) < math.pi / 2
    ratio = ((f + 0.5) / r)[sel]
    assert 0.8 < ratio.mean() < 1.5


# --------------------------------------------------------- mesh distances

def test_point_triangle_golden_cases():
    gold = json.load(open(os.path.join(GOLDEN, "point_triangle.json")))
    a, b, c = (np.array(v, dtype=np.float64) for v in gold["triangle"])
    for case in gold["cases"]:
        q, d2, region = oracle.point_triangle(np.array(case["p"], float), a, b, c)
        assert region == case["region"], case
        assert np.allclose(q, case["q"], atol=1e-15), case
        assert abs(d2 - case["d2"]) < 1e-14, case


def test_point_triangle_against_dense_brute_force():
    """Closest point equals the minimum over a dense barycentric sampling (to sampling error)."""
    rng = np.random.default_rng(21)
    m = 200
    u, v = np.meshgrid(np.linspace(0, 1, m + 1), np.linspace(0, 1, m + 1))
    keep = u + v <= 1
    bary = np.stack([u[keep], v[keep]], 1)
    for _ in range(20):
        a, b, c = rng.normal(size=(3, 3))
        S = a + bary[:, :1] * (b - a) + bary[:, 1:] * (c - a)
        edge = max(np.linalg.norm(b - a), np.linalg.norm(c - a), np.linalg.norm(c - b))
        for p in rng.normal(size=(10, 3)) * 2:
            _, d2, _ = oracle.point_triangle(p, a, b, c)
            dmin = np.min(np.linalg.norm(S - p, axis=1))
            assert math.sqrt(d2) <= dmin + 1e-12
            assert dmin - math.sqrt(d2) <= edge / m


def test_tetrahedron_golden_signed_distances():
    gold = json.load(open(os.path.join(GOLDEN, "tetrahedron.json")))
    V = np.array(gold["vertices"], float)
    F = np.array(gold["faces"], np.int32)
    P = np.array([c["p"] for c in gold["cases"]], float)
    sdf = oracle.mesh_sdf(V, F, P)
    want = np.array([c["sdf"] for c in gold["cases"]])
    assert np.max(np.abs(sdf - want)) < 1e-14


def box_mesh(bx, by, bz):
    V = np.array([[sx * bx, sy * by, sz * bz] for sx in (-1, 1) for sy in (-1, 1) for sz in (-1, 1)],
                 float)
    quads = [(0, 1, 3, 2), (4, 6, 7, 5), (0, 4, 5, 1), (2, 3, 7, 6), (0, 2, 6, 4), (1, 5, 7, 3)]
    F = []
    for a, b, c, d in quads:
        F += [(a, b, c), (a, c, d)]
    F = np.array(F, np.int32)
    # orient outward
    A, B, C = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]
    flip = np.einsum("ij,ij->i", np.cross(B - A, C - A), A + B + C) < 0
    F[flip] = F[flip][:, [0, 2, 1]]
    return V, F


def test_triangulated_box_matches_closed_form_box_sdf():
    b = np.array([0.3, 0.2, 0.4])
    V, F = box_mesh(*b)
    x = I.uniform_points(3000, 13).astype(np.float64)
    q = np.abs(x) - b
    exact = np.linalg.norm(np.maximum(q, 0), axis=1) + np.minimum(q.max(axis=1), 0)
    sdf, w = oracle.mesh_sdf(V, F, x, winding=True)
    assert np.max(np.abs(sdf - exact)) < 1e-14
    inside = exact < 0
    assert np.allclose(w[inside], 1.0, atol=1e-12) and np.allclose(w[~inside], 0.0, atol=1e-12)


def test_icosphere_distance_within_sagitta_of_the_sphere():
    r = 0.5
    V, F = I.icosphere(4, r)
    A, B, C = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]
    nrm = np.cross(B - A, C - A)
    plane = np.abs(np.einsum("ij,ij->i", nrm, A)) / np.linalg.norm(nrm, axis=1)
    sag = r - plane.min()
    x = I.uniform_points(400, 14).astype(np.float64)
    x = x[np.linalg.norm(x, axis=1) > r + 0.01]
    d = oracle.mesh_sdf(V, F, x)
    gap = d - (np.linalg.norm(x, axis=1) - r)
    assert gap.min() >= -1e-12 and gap.max() <= sag + 1e-12


def ray_inside(V, F, x):
    """Inside test for a star-shaped mesh: the ray from the origin through p hits
    one triangle at distance t, and p is inside iff |p| < t (Moller-Trumbore)."""
    A, B, C = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]
    e1, e2 = B - A, C - A
    out = np.empty(len(x), bool)
    for k, p in enumerate(x):
        dvec = p / np.linalg.norm(p)
        pv = np.cross(dvec, e2)
        det = np.einsum("ij,ij->i", e1, pv)
        inv = 1.0 / det
        tv = -A
        u = np.einsum("ij,ij->i", tv, pv) * inv
        qv = np.cross(tv, e1)
        v = (qv @ dvec) * inv
        t = np.einsum("ij,ij->i", e2, qv) * inv
        ok = (u >= 0) & (v >= 0) & (u + v <= 1) & (t > 0)
        out[k] = np.linalg.norm(p) < t[ok].min()
    return out


def test_winding_sign_agrees_with_star_shaped_ray_sign():
    V, F = I.displaced_icosphere(level=3, seed=3)
    x = I.uniform_points(600, 15).astype(np.float64) * 0.7
    sdf, w = oracle.mesh_sdf(V, F, x, winding=True)
    assert np.array_equal(sdf < 0, ray_inside(V, F, x))
    assert np.all(np.minimum(np.abs(w), np.abs(w - 1)) < 1e-9)


# ----------------------------------------------------------------- fitting

def torch_fit_loss(spec, params, x, s, delta):
    P = torch.tensor(np.asarray(params, np.float64), requires_grad=True)
    X = torch.tensor(np.asarray(x, np.float64))
    off, h = 0, X
    shapes = I.layer_shapes(spec)
    for l, (o, i) in enumerate(shapes[:-1], start=1):
        W = P[off:off + o * i].view(o, i)
        off += o * i
        b = P[off:off + o]
        off += o
        u = torch.cat([h, X], 1) if l == spec.skip else h
        h = torch.nn.functional.softplus(u @ W.T + b, beta=spec.beta, threshold=30.0)
    _, i = shapes[-1]
    f = h @ P[off:off + i] + P[off + i]
    S = torch.tensor(np.asarray(s, np.float64))
    loss = (f.clamp(-delta, delta) - S.clamp(-delta, delta)).abs().mean()
    (g,) = torch.autograd.grad(loss, P)
    return float(loss), g.numpy()


def test_fit_loss_gradient_matches_torch_and_differences():
    spec, params = random_net(8, (24, 24, 24, 24), 3, scale=1.0)
    x = I.uniform_points(400, 16) * 0.5
    s = np.linalg.norm(x.astype(np.float64), axis=1) - 0.3
    delta = 0.1
    loss, g = oracle.fit_loss(spec, params, x, s, delta)
    lt, gt = torch_fit_loss(spec, params, x, s, delta)
    assert abs(loss - lt) < 1e-14
    assert np.max(np.abs(g - gt)) < 1e-13
    # central differences on a few parameters (the loss is piecewise smooth)
    rng = np.random.default_rng(0)
    P = params.astype(np.float64)
    for k in rng.choice(P.size, 24, replace=False):
        h = 1e-7
        Pp, Pm = P.copy(), P.copy()
        Pp[k] += h
        Pm[k] -= h
        fd = (oracle.fit_loss(spec, Pp, x, s, delta)[0] - oracle.fit_loss(spec, Pm, x, s, delta)[0]) / (2 * h)
        assert abs(fd - g[k]) < 1e-6 * (1 + abs(g[k]))
