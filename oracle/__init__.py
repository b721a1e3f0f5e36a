"""FP64 CPU oracle for neural-SDF collision handling -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library and
its binding) never imports, links or calls anything here, and this package
imports nothing from the product.  It wraps ``sdf_oracle.c`` (plain C, FP64,
OpenMP) with ctypes; see that file for the passage of the paper each function
follows.

Inputs are numpy arrays; parameters and points are typically the float32
arrays drawn by the seeded input generators and are widened to float64 here.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sdf_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# Test hook: the mutation tests point this at a deliberately broken build.
_OVERRIDE = os.environ.get("SDF_ORACLE_LIB")
_lib = None

_f64p = ctypes.POINTER(ctypes.c_double)
_i32p = ctypes.POINTER(ctypes.c_int32)
_u8p = ctypes.POINTER(ctypes.c_uint8)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (strict ISO C, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-std=c11", "-O2", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        path = _OVERRIDE or _LIB
        if not _OVERRIDE and (not os.path.exists(_LIB)
                              or os.path.getmtime(_LIB) < os.path.getmtime(_SRC)):
            build()
        lib = ctypes.CDLL(path)
        lib.orc_param_count.restype = ctypes.c_int64
        lib.orc_param_count.argtypes = [ctypes.c_int, _i32p, ctypes.c_int]
        for name in ("orc_mlp_eval", "orc_mlp_jvp"):
            fn = getattr(lib, name)
            fn.restype = ctypes.c_int
            fn.argtypes = [ctypes.c_int, _i32p, ctypes.c_int, ctypes.c_double, _f64p,
                           ctypes.c_int64, _f64p, _f64p, _f64p]
        lib.orc_collide.restype = None
        lib.orc_collide.argtypes = [ctypes.c_int64, _f64p, _f64p, _f64p, ctypes.c_double,
                                    _f64p, _f64p, _u8p]
        lib.orc_point_tri.restype = ctypes.c_int
        lib.orc_point_tri.argtypes = [_f64p, _f64p, _f64p, _f64p, _f64p, _f64p]
        lib.orc_solid_angle.restype = ctypes.c_double
        lib.orc_solid_angle.argtypes = [_f64p, _f64p, _f64p, _f64p]
        lib.orc_mesh_sdf.restype = None
        lib.orc_mesh_sdf.argtypes = [ctypes.c_int64, _f64p, ctypes.c_int64, _i32p,
                                     ctypes.c_int64, _f64p, _f64p, _f64p]
        lib.orc_fit_loss.restype = ctypes.c_int
        lib.orc_fit_loss.argtypes = [ctypes.c_int, _i32p, ctypes.c_int, ctypes.c_double, _f64p,
                                     ctypes.c_int64, _f64p, _f64p, ctypes.c_double, _f64p, _f64p]
        _lib = lib
    return _lib


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a, t=_f64p):
    return None if a is None else a.ctypes.data_as(t)


def _net(spec):
    w = np.ascontiguousarray(spec.widths, dtype=np.int32)
    return len(spec.widths), w, int(spec.skip), float(spec.beta)


def param_count(spec) -> int:
    if getattr(spec, "fourier", 0):
        from . import fourier
        prev, n = 2 * spec.fourier, 3 * spec.fourier
        for w in spec.widths:
            n += w * prev + w
            prev = w
        return n + prev + 1
    L, w, skip, _ = _net(spec)
    return int(_load().orc_param_count(L, _p(w, _i32p), skip))


def mlp_eval(spec, params, pts, grad: bool = True, mode: str = "reverse"):
    """f (n,) and, if grad, the input gradient (n,3) in float64.

    mode "reverse" back-propagates (Sec. 3.2); "forward" propagates tangents.
    """
    if getattr(spec, "fourier", 0):  # Fourier-feature input (numpy, oracle/fourier.py)
        from . import fourier
        return fourier.mlp_eval(spec, params, pts, grad)
    L, w, skip, beta = _net(spec)
    P, X = _d(params), _d(pts).reshape(-1, 3)
    if P.size != param_count(spec):
        raise ValueError("params has %d values, expected %d" % (P.size, param_count(spec)))
    n = X.shape[0]
    f = np.empty(n)
    g = np.empty((n, 3)) if grad else None
    fn = _load().orc_mlp_eval if mode == "reverse" else _load().orc_mlp_jvp
    rc = fn(L, _p(w, _i32p), skip, beta, _p(P), n, _p(X), _p(f), _p(g))
    if rc != 0:
        raise RuntimeError("oracle mlp failed: %d" % rc)
    return (f, g) if grad else f


def collide(pts, f, grad, eps: float):
    """Projected points, unit normals and hit flags (Eq. 2, Eq. 3)."""
    X = _d(pts).reshape(-1, 3)
    n = X.shape[0]
    F, G = _d(f).reshape(n), _d(grad).reshape(n, 3)
    out, nrm = np.empty((n, 3)), np.empty((n, 3))
    hit = np.empty(n, dtype=np.uint8)
    _load().orc_collide(n, _p(X), _p(F), _p(G), float(eps), _p(out), _p(nrm), _p(hit, _u8p))
    return out, nrm, hit


def collide_project(spec, params, pts, eps: float):
    """The whole path in FP64: f, grad f, normal, hit and moved points."""
    f, g = mlp_eval(spec, params, pts)
    out, nrm, hit = collide(pts, f, g, eps)
    return {"sdf": f, "grad": g, "normal": nrm, "hit": hit, "pts": out}


def collide_project_rigid(spec, params, pts, eps: float, T):
    """The path for a collider placed in the world by T = [A t; 0 1] (Sec. 4.2):
    the network is evaluated at p' = A^{-1}(p - t), the gradient of
    p -> f(A^{-1}(p - t)) is A^{-T} grad f(p') (for a rotation A: A grad f(p'),
    the rotated normal of Sec. 4.2), and the vertex moves in the world frame."""
    T = _d(T).reshape(4, 4)
    A, t = T[:3, :3], T[:3, 3]
    X = _d(pts).reshape(-1, 3)
    local = np.linalg.solve(A, (X - t).T).T
    f, gl = mlp_eval(spec, params, local)
    g = np.linalg.solve(A.T, gl.T).T
    out, nrm, hit = collide(X, f, g, eps)
    return {"sdf": f, "grad": g, "normal": nrm, "hit": hit, "pts": out}


def point_triangle(p, a, b, c):
    """(closest point, squared distance, Voronoi region id) for one triangle."""
    q, d2 = np.empty(3), np.empty(1)
    r = _load().orc_point_tri(_p(_d(p)), _p(_d(a)), _p(_d(b)), _p(_d(c)), _p(q), _p(d2))
    return q, float(d2[0]), int(r)


def solid_angle(p, a, b, c) -> float:
    return float(_load().orc_solid_angle(_p(_d(p)), _p(_d(a)), _p(_d(b)), _p(_d(c))))


def mesh_sdf(V, F, pts, winding: bool = False):
    """Brute-force signed distance of every point to a closed triangle mesh."""
    V, X = _d(V).reshape(-1, 3), _d(pts).reshape(-1, 3)
    T = np.ascontiguousarray(F, dtype=np.int32).reshape(-1, 3)
    n = X.shape[0]
    sdf, wind = np.empty(n), (np.empty(n) if winding else None)
    _load().orc_mesh_sdf(V.shape[0], _p(V), T.shape[0], _p(T, _i32p), n, _p(X), _p(sdf), _p(wind))
    return (sdf, wind) if winding else sdf


def fit_loss(spec, params, pts, targets, delta: float = 0.1):
    """Clamped-L1 loss and its gradient w.r.t. the flat parameters (FP64)."""
    L, w, skip, beta = _net(spec)
    P, X, S = _d(params), _d(pts).reshape(-1, 3), _d(targets).ravel()
    g = np.empty(P.size)
    loss = np.empty(1)
    rc = _load().orc_fit_loss(L, _p(w, _i32p), skip, beta, _p(P), X.shape[0], _p(X), _p(S),
                              float(delta), _p(loss), _p(g))
    if rc != 0:
        raise RuntimeError("oracle fit_loss failed: %d" % rc)
    return float(loss[0]), g
