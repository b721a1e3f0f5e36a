"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances:
  FP32 operands: |f - f64| <= 1e-5 (1 + |f64|), angle(grad, grad64) <= 1e-4 rad.
  BF16 / FP16 operands: the stated accuracy target, |f - f64| <= 1e-3 and
  normal angle <= 1e-2 rad (max over all points), asserted where each test
  says so; the measured statistics are always printed.
  FP8 (E4M3) operands, no target is stated; the bound comes from the
  arithmetic: 3 mantissa bits (unit roundoff 2^-4) on both operands of every
  hidden contraction.  The operand-rounding model of tests/precision_model.py
  gives, on geometric-init nets of widths 256 and 512 (2048 uniform points),
  |f - f64| <= 0.089 and normal angles with p99 <= 0.103 and max <= 0.153 rad
  (tests/test_precision_model.py::test_fp8_error_bound_of_the_gpu_tests); the
  tests assert |f - f64| <= 0.15, p99 angle <= 0.15 and max angle <= 0.6 rad.
Hits are decided in FP32 on both sides of the comparison that must be exact:
the GPU's flag equals (its own f < eps); against FP64 the flags agree wherever
|f64 - eps| exceeds the SDF tolerance.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from paper_2110_01614_amd import inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - collected on CPU machines
    pytest.skip("needs a GPU", allow_module_level=True)

B = pytest.importorskip("paper_2110_01614_amd.binding")

STATS = os.environ.get("SDF_STATS_OUT")
TOL = {"fp32": (1e-5, 1e-4), "bf16": (1e-3, 1e-2), "fp16": (1e-3, 1e-2), "bf16x3": (1e-3, 1e-2),
       "fp8": (0.15, 0.6)}
# precisions whose accuracy target is asserted on every workload
GATED = ("fp32", "bf16x3")


def angle(a, b):
    cr = np.linalg.norm(np.cross(a, b), axis=1)
    return np.arctan2(cr, np.einsum("ij,ij->i", a, b))


def record(name, **kv):
    line = json.dumps(dict(test=name, **kv))
    print(line, flush=True)
    if STATS:
        with open(STATS, "a") as fh:
            fh.write(line + "\n")


def run_gpu(spec, params, pts, precision, eps=0.005):
    net = B.SdfNet(spec, params, precision)
    X = torch.from_numpy(np.ascontiguousarray(pts, np.float32)).cuda()
    fq = net.query(X)
    fg, g = net.query_grad(X)
    P = X.clone()
    outs = net.collide_project(P, eps)
    torch.cuda.synchronize()
    res = dict(fq=fq.cpu().numpy(), fg=fg.cpu().numpy(), grad=g.cpu().numpy(), pts=P.cpu().numpy(),
               sdf=outs["sdf"].cpu().numpy(), normal=outs["normal"].cpu().numpy(),
               hit=outs["hit"].cpu().numpy())
    net.close()
    return res


def compare(name, spec, params, pts, precision, eps=0.005, assert_gate=True, ref=None):
    pts = np.ascontiguousarray(pts, np.float32)
    ref = ref or oracle.collide_project(spec, params, pts, eps)
    got = run_gpu(spec, params, pts, precision, eps)
    tol_f, tol_a = TOL[precision]
    f64 = ref["sdf"]
    # all three entry points agree on f
    assert np.array_equal(got["fq"], got["fg"]) and np.array_equal(got["fg"], got["sdf"])
    ferr = np.abs(got["fg"] - f64)
    gn = np.linalg.norm(ref["grad"], axis=1)
    ok = gn > 1e-6 * np.median(gn)
    ang = angle(got["grad"][ok].astype(np.float64), ref["grad"][ok])
    nang = angle(got["normal"][ok].astype(np.float64), ref["normal"][ok])
    record(name, precision=precision, n=len(pts), sdf_max=float(ferr.max()),
           sdf_p99=float(np.quantile(ferr, 0.99)), sdf_mean=float(ferr.mean()),
           ang_max=float(ang.max()), ang_p99=float(np.quantile(ang, 0.99)), ang_mean=float(ang.mean()),
           f_range=[float(f64.min()), float(f64.max())])
    # hit flag: exact against the GPU's own f, and against FP64 away from the threshold
    assert np.array_equal(got["hit"].astype(bool), got["sdf"] < np.float32(eps))
    far = np.abs(f64 - eps) > 2 * tol_f * (1 + np.abs(f64))
    assert np.array_equal(got["hit"][far].astype(bool), ref["hit"][far].astype(bool))
    # vertices that are not hit keep their exact bits
    miss = got["hit"] == 0
    assert np.array_equal(got["pts"][miss].view(np.uint32), pts[miss].view(np.uint32))
    # the normal is the normalised gradient of the same call
    gg = got["grad"].astype(np.float64)
    nn = gg / np.linalg.norm(gg, axis=1, keepdims=True)
    assert np.max(np.abs(nn[ok] - got["normal"][ok])) < 1e-5
    if precision in GATED or assert_gate:
        if precision == "fp32":
            assert np.all(ferr <= tol_f * (1 + np.abs(f64)))
        else:
            assert ferr.max() <= tol_f
        assert ang.max() <= tol_a
        # moved vertices: p + (eps - f) N within the propagated tolerance
        both = (got["hit"] == 1) & (ref["hit"] == 1) & ok
        dp = np.linalg.norm(got["pts"][both] - ref["pts"][both], axis=1)
        bound = tol_f * (1 + np.abs(f64[both])) + np.abs(eps - f64[both]) * tol_a * 1.01 + \
            4e-7 * (1 + np.linalg.norm(pts[both], axis=1))
        assert np.all(dp <= bound)
    return got, ref


def random_net(seed, widths, skip, scale=1.0):
    spec = I.NetSpec(tuple(widths), skip=skip)
    rng = np.random.default_rng(seed)
    parts = []
    for o, i in I.layer_shapes(spec):
        parts.append(rng.normal(0, scale / math.sqrt(i), size=o * i))
        parts.append(rng.normal(0, 0.01, size=o))
    return spec, np.concatenate(parts).astype(np.float32)


# ------------------------------------------------------------------ workloads

@pytest.mark.parametrize("precision", ["fp32", "bf16", "fp16", "bf16x3"])
def test_sphere64_all_points(precision):
    """3->64x3->1 geometric sphere net, all 4096 uniform points."""
    spec, params, pts, eps = I.workload_inputs("sphere64")
    compare("sphere64", spec, params, pts, precision, eps, assert_gate=False)


@pytest.mark.parametrize("precision", ["fp32", "bf16", "fp16", "bf16x3"])
@pytest.mark.parametrize("init", ["normal", "geometric"])
def test_cloth_net_on_cloth_subset(precision, init):
    """3->256x8->1 skip-5 net on 3000 cloth vertices (46 full tiles + ragged)."""
    spec, params, pts, eps = I.workload_inputs("cloth1m", init=init)
    idx = np.random.default_rng(9).choice(len(pts), 3000, replace=False)
    compare("cloth_subset_" + init, spec, params, pts[idx], precision, eps, assert_gate=False)


SHAPES = [((64, 64), 0), ((64,) * 5, 3), ((128, 128, 128), 2), ((128,) * 8, 8),
          ((256, 256), 2), ((256,) * 4, 0), ((256,) * 6, 4), ((64,) * 8, 5), ((512,) * 3, 2),
          ((512,) * 8, 5)]


@pytest.mark.parametrize("widths,skip", SHAPES)
@pytest.mark.parametrize("precision", ["fp32", "bf16", "bf16x3"])
def test_shapes_and_ragged_sizes(widths, skip, precision):
    if widths[0] == 512 and precision == "fp32":
        pytest.skip("width 512 has 16-bit kernels only")
    spec, params = random_net(hash((widths, skip)) % 1000, widths, skip)
    for n in (1, 17, 64, 1000):
        pts = I.uniform_points(n, n)
        compare("shape_%dx%d_s%d_n%d" % (widths[0], len(widths), skip, n), spec, params, pts,
                precision, assert_gate=False)


def test_cloth_full_size_sampled():
    """The full 1M-vertex cloth in the benchmark's launch shape, 4096 sampled outputs."""
    spec, params, pts, eps = I.workload_inputs("cloth1m")
    idx = np.random.default_rng(3).choice(len(pts), 4096, replace=False)
    ref = oracle.collide_project(spec, params, pts[idx], eps)
    for precision in ("fp32", "bf16", "fp16", "bf16x3"):
        got = run_gpu(spec, params, pts, precision, eps)
        ferr = np.abs(got["fg"][idx] - ref["sdf"])
        ang = angle(got["grad"][idx].astype(np.float64), ref["grad"])
        record("cloth1m_sampled", precision=precision, sdf_max=float(ferr.max()),
               ang_max=float(ang.max()), ang_p99=float(np.quantile(ang, 0.99)))
        tol_f, tol_a = TOL[precision]
        assert ferr.max() <= tol_f * (1 + np.abs(ref["sdf"]).max())
        if precision in GATED:
            assert ang.max() <= tol_a
        assert np.array_equal(got["hit"].astype(bool), got["sdf"] < np.float32(eps))


def fp8_check(name, got, ref):
    ferr = np.abs(got["fg"].astype(np.float64) - ref["sdf"])
    gn = np.linalg.norm(ref["grad"], axis=1)
    ok = gn > 1e-6 * np.median(gn)
    ang = angle(got["grad"][ok].astype(np.float64), ref["grad"][ok])
    record(name + "_fp8_check", sdf_max=float(ferr.max()), ang_p99=float(np.quantile(ang, 0.99)),
           ang_max=float(ang.max()))
    tol_f, tol_a = TOL["fp8"]
    assert ferr.max() <= tol_f
    assert np.quantile(ang, 0.99) <= 0.15 and ang.max() <= tol_a


FP8_SHAPES = [((128,) * 4, 2), ((256,) * 8, 5), ((512,) * 3, 2), ((512,) * 8, 5)]


@pytest.mark.parametrize("widths,skip", FP8_SHAPES)
def test_fp8_shapes_geometric(widths, skip):
    """E4M3 operands on geometric-init nets, 1 / 17 / 100 / 1000 points."""
    spec = I.NetSpec(tuple(widths), skip=skip)
    params = I.init_geometric(spec, 3)
    for n in (1, 17, 100, 1000):
        pts = I.uniform_points(n, 40 + n)
        name = "fp8_%dx%d_s%d_n%d" % (widths[0], len(widths), skip, n)
        got, ref = compare(name, spec, params, pts, "fp8", assert_gate=False)
        fp8_check(name, got, ref)


def test_wide_net_4m_points_sampled():
    """3->512x8->1 skip 5, 4M uniform points in the benchmark's launch shape:
    BF16, BF16x3 and FP8 on 4096 sampled outputs against FP64."""
    spec, params, pts, eps = I.workload_inputs("wide4m")
    idx = np.random.default_rng(4).choice(len(pts), 4096, replace=False)
    ref = oracle.collide_project(spec, params, pts[idx], eps)
    for precision in ("bf16", "bf16x3", "fp8"):
        got = run_gpu(spec, params, pts, precision, eps)
        sub = {k: v[idx] for k, v in got.items()}
        ferr = np.abs(sub["fg"] - ref["sdf"])
        ang = angle(sub["grad"].astype(np.float64), ref["grad"])
        record("wide4m_sampled", precision=precision, sdf_max=float(ferr.max()),
               ang_max=float(ang.max()), ang_p99=float(np.quantile(ang, 0.99)))
        assert np.array_equal(got["hit"].astype(bool), got["sdf"] < np.float32(eps))
        if precision == "bf16x3":
            assert ferr.max() <= TOL["bf16x3"][0] and ang.max() <= TOL["bf16x3"][1]
        if precision == "fp8":
            fp8_check("wide4m", sub, ref)


def rotation(seed):
    q = np.random.default_rng(seed).normal(size=4)
    w, x, y, z = q / np.linalg.norm(q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                     [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                     [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


@pytest.mark.parametrize("precision", ["fp32", "bf16", "bf16x3", "fp8"])
def test_rigid_frame(precision):
    """A collider moved by T = [R t; 0 1] (Sec. 4.2) against the FP64 oracle;
    the identity frame reproduces the plain calls bit for bit."""
    spec = I.NetSpec((256,) * 4, skip=2)
    params = I.init_geometric(spec, 6)
    T = np.eye(4)
    T[:3, :3], T[:3, 3] = rotation(8), [0.25, -0.1, 0.05]
    pts = (I.uniform_points(3000, 15) * 0.9 + T[:3, 3]).astype(np.float32)
    eps = 0.005
    ref = oracle.collide_project_rigid(spec, params, pts, eps, T)
    net = B.SdfNet(spec, params, precision)
    X = torch.from_numpy(pts).cuda()
    fq = net.query(X, T=T)
    fg, g = net.query_grad(X, T=T)
    P = X.clone()
    outs = net.collide_project(P, eps, T=T)
    # identity frame == plain entry points
    I4 = np.eye(4)
    f_id, g_id = net.query_grad(X, T=I4)
    f_pl, g_pl = net.query_grad(X)
    torch.cuda.synchronize()
    assert torch.equal(f_id, f_pl) and torch.equal(g_id, g_pl)
    fq, fg, g = fq.cpu().numpy(), fg.cpu().numpy(), g.cpu().numpy().astype(np.float64)
    P, hit = P.cpu().numpy(), outs["hit"].cpu().numpy()
    assert np.array_equal(fq, fg) and np.array_equal(fg, outs["sdf"].cpu().numpy())
    ferr = np.abs(fg - ref["sdf"])
    ang = angle(g, ref["grad"])
    record("rigid_frame", precision=precision, sdf_max=float(ferr.max()), ang_max=float(ang.max()),
           ang_p99=float(np.quantile(ang, 0.99)))
    assert np.array_equal(hit.astype(bool), fg < np.float32(eps))
    miss = hit == 0
    assert np.array_equal(P[miss].view(np.uint32), pts[miss].view(np.uint32))
    tol_f, tol_a = TOL[precision]
    if precision == "fp32":
        assert np.all(ferr <= tol_f * (1 + np.abs(ref["sdf"]))) and ang.max() <= tol_a
    elif precision == "bf16x3":
        assert ferr.max() <= tol_f and ang.max() <= tol_a
    elif precision == "fp8":
        fp8_check("rigid", {"fg": fg, "grad": g}, ref)
    if precision in ("fp32", "bf16x3"):  # moved vertices in the world frame
        both = (hit == 1) & (ref["hit"] == 1)
        dp = np.linalg.norm(P[both] - ref["pts"][both], axis=1)
        assert np.all(dp <= tol_f * (1 + np.abs(ref["sdf"][both])) + np.abs(eps - ref["sdf"][both]) * tol_a
                      + 1e-6)
    with pytest.raises(B.SdfError):
        net.query(X, T=np.zeros((4, 4)))  # singular, bad last row
    net.close()


FF_SHAPES = [((128,) * 4, 64), ((256,) * 4, 128), ((256,) * 8, 128)]


@pytest.mark.parametrize("precision", ["bf16", "fp16", "bf16x3"])
@pytest.mark.parametrize("widths,m", FF_SHAPES)
def test_fourier_features(widths, m, precision):
    """Fourier-feature input (Sec. 3.1, Sec. 4.3; the timed nets are 256 x 4 and
    256 x 8): layer 1 runs on MFMA over gamma(x), and the reverse sweep continues
    through the mapping.  1000 points (15 full tiles and a ragged one) and 17."""
    spec = I.NetSpec(tuple(widths), fourier=m)
    params = I.init_fourier(spec, 11, 2.0)
    for n in (17, 1000):
        pts = I.uniform_points(n, 21 + n)
        compare("fourier_%dx%d_n%d" % (widths[0], len(widths), n), spec, params, pts, precision,
                assert_gate=precision == "bf16x3")


# ------------------------------------------------------------- exact cases

def plane_net(n, d, C=2.5, widths=(64,) * 6, skip=4, seed=5):
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
    return spec, np.concatenate(parts).astype(np.float32)


def test_plane_net_projects_onto_the_plane_fp32():
    """An MLP that is exactly the plane n.x - d (closed form, no oracle)."""
    n = np.array([0.6, -0.48, 0.64], np.float32)
    d, eps = 0.25, 0.01
    spec, params = plane_net(n, d)
    pts = I.uniform_points(5000, 31)
    got = run_gpu(spec, params, pts, "fp32", eps)
    exact = pts.astype(np.float64) @ n.astype(np.float64) - d
    assert np.max(np.abs(got["fg"] - exact)) < 2e-6
    assert np.max(np.abs(got["grad"] - n)) < 1e-6
    hit = got["hit"] == 1
    f2 = got["pts"][hit].astype(np.float64) @ n.astype(np.float64) - d
    assert np.max(np.abs(f2 - eps)) < 3e-6


@pytest.mark.parametrize("precision", ["fp32", "bf16", "fp16", "bf16x3", "fp8"])
def test_nan_vertex_is_not_moved_and_bits_kept(precision):
    """A NaN vertex has f = NaN, is never a hit and keeps its bits; the others
    are unaffected (FP8 runs on a width-128 net, its narrowest)."""
    if precision == "fp8":
        spec = I.NetSpec((128,) * 4)
        params, pts, eps = I.init_geometric(spec, 0), I.uniform_points(100, 1), 0.005
    else:
        spec, params, pts, eps = I.workload_inputs("sphere64", n=100)
    clean = run_gpu(spec, params, pts, precision, eps)
    pts = pts.copy()
    pts[7] = np.nan
    pts[40, 1] = np.nan  # one NaN coordinate is enough
    got = run_gpu(spec, params, pts, precision, eps)
    for i in (7, 40):
        assert np.isnan(got["sdf"][i]) and got["hit"][i] == 0
        assert np.array_equal(got["pts"][i].view(np.uint32), pts[i].view(np.uint32))
    rest = np.ones(len(pts), bool)
    rest[[7, 40]] = False
    assert np.array_equal(got["sdf"][rest], clean["sdf"][rest])
    assert np.array_equal(got["pts"][rest], clean["pts"][rest])


def test_argument_errors_and_empty_input():
    spec, params, pts, eps = I.workload_inputs("sphere64", n=64)
    net = B.SdfNet(spec, params, "fp32")
    X = torch.from_numpy(pts).cuda()
    out = torch.empty(64, device="cuda")
    assert B.lib.sdf_query(net.handle, X.data_ptr(), 0, out.data_ptr(), None) == B.SDF_OK
    assert B.lib.sdf_query(net.handle, X.data_ptr(), -1, out.data_ptr(), None) == B.SDF_EINVAL
    assert B.lib.sdf_query(net.handle, None, 64, out.data_ptr(), None) == B.SDF_EINVAL
    assert B.lib.sdf_query(net.handle, X.data_ptr(), 64, None, None) == B.SDF_EINVAL
    assert B.lib.sdf_query(net.handle, X.data_ptr() + 2, 64, out.data_ptr(), None) == B.SDF_EINVAL
    assert B.lib.sdf_query_grad(net.handle, X.data_ptr(), 64, None, None, None) == B.SDF_EINVAL
    assert B.lib.collide_project(net.handle, X.data_ptr(), 64, float("nan"), None, None, None,
                                 None) == B.SDF_EINVAL
    torch.cuda.synchronize()
    net.close()


def test_repeatable_bits_and_side_stream():
    spec, params, pts, eps = I.workload_inputs("cloth1m")
    pts = pts[:20000]
    net = B.SdfNet(spec, params, "bf16")
    X = torch.from_numpy(pts).cuda()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        a = net.query_grad(X)
        b = net.query_grad(X)
    s.synchronize()
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    c = net.query_grad(X)
    torch.cuda.synchronize()
    assert torch.equal(a[1], c[1])
    net.close()


def test_fp32_handle_on_two_streams_is_ordered():
    """FP32 handles keep one reverse-sweep scratch area: calls issued back to
    back on two streams are ordered on the device by the library, so each
    result equals its serial run bit for bit and the FP64 oracle within the
    FP32 tolerance.  20,000 points = 313 tiles: every scratch slot is used."""
    spec, params, pts, eps = I.workload_inputs("cloth1m", init="geometric")
    p1, p2 = np.ascontiguousarray(pts[:20000]), np.ascontiguousarray(pts[500000:520000])
    net = B.SdfNet(spec, params, "fp32")
    X1, X2 = torch.from_numpy(p1).cuda(), torch.from_numpy(p2).cuda()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    for _ in range(3):
        with torch.cuda.stream(s1):
            a = net.query_grad(X1)
        with torch.cuda.stream(s2):
            b = net.query_grad(X2)
        torch.cuda.synchronize()
    a_ser = net.query_grad(X1)
    torch.cuda.synchronize()
    b_ser = net.query_grad(X2)
    torch.cuda.synchronize()
    assert torch.equal(a[0], a_ser[0]) and torch.equal(a[1], a_ser[1])
    assert torch.equal(b[0], b_ser[0]) and torch.equal(b[1], b_ser[1])
    for P, (f, g) in ((p1, a), (p2, b)):
        f64, g64 = oracle.mlp_eval(spec, params, P)
        f, g = f.cpu().numpy(), g.cpu().numpy().astype(np.float64)
        assert np.all(np.abs(f - f64) <= 1e-5 * (1 + np.abs(f64)))
        assert angle(g, g64).max() <= 1e-4
    net.close()


# The stated accuracy target on the cloth workload's two networks: met or
# missed per precision exactly as the operand-rounding model predicts
# (tests/test_precision_model.py): plain BF16 misses it on both, FP16 misses
# the angle bar on the N(0, 0.02) net and meets both bars on the geometric
# one, BF16x3 meets both on both.
TARGET_CASES = [("bf16", "normal", False), ("bf16", "geometric", False), ("fp16", "normal", False),
                ("fp16", "geometric", True), ("bf16x3", "normal", True), ("bf16x3", "geometric", True)]


@pytest.mark.parametrize("precision,init,meets", TARGET_CASES)
def test_accuracy_target_on_the_cloth_networks(precision, init, meets):
    """Max |f - f64| <= 1e-3 and max normal angle <= 1e-2 rad over 4096 cloth
    vertices, through query_grad."""
    spec, params, pts, eps = I.workload_inputs("cloth1m", init=init)
    P = np.ascontiguousarray(pts[np.random.default_rng(3).choice(len(pts), 4096, replace=False)])
    f64, g64 = oracle.mlp_eval(spec, params, P)
    net = B.SdfNet(spec, params, precision)
    f, g = net.query_grad(torch.from_numpy(P).cuda())
    torch.cuda.synchronize()
    f, g = f.cpu().numpy().astype(np.float64), g.cpu().numpy().astype(np.float64)
    net.close()
    ferr, ang = np.abs(f - f64).max(), angle(g, g64).max()
    record("accuracy_target", precision=precision, init=init, sdf_max=float(ferr), ang_max=float(ang))
    within = ferr <= 1e-3 and ang <= 1e-2
    assert within == meets, (precision, init, ferr, ang)


@pytest.mark.parametrize("precision", ["fp32", "bf16", "fp16", "bf16x3"])
def test_zero_gradient_hit_is_not_moved(precision):
    """A network whose output weights are zero: f = b_o < eps everywhere and
    grad f = 0 exactly, so every vertex is a hit, its normal is 0 and it is
    not moved (bits kept)."""
    spec = I.NetSpec((128,) * 4, 2)
    params = np.zeros(I.param_count(spec), np.float32)
    params[-1] = -0.1
    pts = I.uniform_points(777, 40)
    got = run_gpu(spec, params, pts, precision, 0.005)
    assert np.all(got["hit"] == 1)
    assert np.all(got["sdf"] == np.float32(-0.1))
    assert np.all(got["grad"] == 0.0) and np.all(got["normal"] == 0.0)
    assert np.array_equal(got["pts"].view(np.uint32), pts.view(np.uint32))


@pytest.mark.parametrize("nth", [1, 2, 3])
def test_device_allocation_failure_is_reported(nth, monkeypatch):
    """SDFC_FAIL_ALLOC=k makes the k-th device allocation of sdf_net_create
    fail: the call returns SDF_ENOMEM and leaves nothing behind."""
    spec, params, pts, eps = I.workload_inputs("sphere64", n=64)
    d = B.make_desc(spec.widths, spec.skip, precision="fp32")
    monkeypatch.setenv("SDFC_FAIL_ALLOC", str(nth))
    with pytest.raises(B.SdfError) as e:
        B.sdf_net_create(d, params)
    assert e.value.code == B.SDF_ENOMEM
    monkeypatch.delenv("SDFC_FAIL_ALLOC")
    h = B.sdf_net_create(d, params)
    B.sdf_net_destroy(h)
