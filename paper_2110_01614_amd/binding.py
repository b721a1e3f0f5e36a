"""Thin ctypes binding of libsdfcollide.so (declared in include/sdfcollide.h).

Argument marshalling only: every step of the path runs in the HIP kernels.
Functions keep the C names; ``SdfNet`` is a small owner of a handle that
takes torch CUDA tensors (PyTorch supplies device memory and the stream).
Importing this module loads the library and raises if it is missing -- there
is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsdfcollide.so")

SDF_OK, SDF_EINVAL, SDF_EUNSUPPORTED, SDF_ENOMEM, SDF_EDEVICE = 0, -1, -2, -3, -4
SDF_FP32, SDF_BF16, SDF_FP16, SDF_BF16X3, SDF_FP8 = 0, 1, 2, 3, 4
SDF_MAX_HIDDEN = 16
SDF_GROUP_PER_WIDTH, SDF_GROUP_PER_NETWORK, SDF_GROUP_PERSISTENT = 0, 1, 2
GROUP_MODES = {"per_width": SDF_GROUP_PER_WIDTH, "per_network": SDF_GROUP_PER_NETWORK,
               "persistent": SDF_GROUP_PERSISTENT}
PRECISIONS = {"fp32": SDF_FP32, "bf16": SDF_BF16, "fp16": SDF_FP16, "bf16x3": SDF_BF16X3, "fp8": SDF_FP8}


class sdf_net_desc(ctypes.Structure):
    _fields_ = [("n_hidden", ctypes.c_int32),
                ("width", ctypes.c_int32 * SDF_MAX_HIDDEN),
                ("skip_layer", ctypes.c_int32),
                ("beta", ctypes.c_float),
                ("precision", ctypes.c_int32),
                ("fourier", ctypes.c_int32)]


class SdfError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("sdfcollide error %d: %s" % (code, msg))
        self.code = code


def _hip_runtimes_mapped():
    """Distinct files of the HIP runtime (libamdhip64) mapped into this process."""
    found = set()
    try:
        with open("/proc/self/maps") as f:
            for line in f:
                path = line.split()[-1] if "/" in line else ""
                if os.path.basename(path).startswith("libamdhip64.so"):
                    found.add(os.path.realpath(path))
    except OSError:
        pass
    return found


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libsdfcollide.so is not built (run paper_2110_01614_amd.build); "
                          "there is no fallback implementation")
    # PyTorch supplies device memory and streams, so the library must share its
    # HIP runtime.  torch ships its own libamdhip64 (soname libamdhip64.so.7)
    # and its libraries ask for it by another name; if this library were loaded
    # first, the system copy it needs would come in under that soname and torch
    # would then map its own copy beside it -- two runtimes, and the second one
    # to initialise sees no device.  Loading torch first makes this library's
    # dependency resolve to the runtime already in the process.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    runtimes = _hip_runtimes_mapped()
    if len(runtimes) > 1:
        raise ImportError("more than one HIP runtime is mapped into this process (%s); load "
                          "libsdfcollide.so only after torch" % ", ".join(sorted(runtimes)))
    vp, i64, f32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_float
    desc_p = ctypes.POINTER(sdf_net_desc)
    lib.sdf_param_count.restype = i64
    lib.sdf_param_count.argtypes = [desc_p]
    lib.sdf_net_create.restype = ctypes.c_int
    lib.sdf_net_create.argtypes = [desc_p, ctypes.POINTER(ctypes.c_float), ctypes.c_size_t,
                                   ctypes.c_int, ctypes.POINTER(vp)]
    lib.sdf_net_destroy.restype = ctypes.c_int
    lib.sdf_net_destroy.argtypes = [vp]
    lib.sdf_query.restype = ctypes.c_int
    lib.sdf_query.argtypes = [vp, vp, i64, vp, vp]
    lib.sdf_query_grad.restype = ctypes.c_int
    lib.sdf_query_grad.argtypes = [vp, vp, i64, vp, vp, vp]
    lib.collide_project.restype = ctypes.c_int
    lib.collide_project.argtypes = [vp, vp, i64, f32, vp, vp, vp, vp]
    lib.sdf_last_error.restype = ctypes.c_char_p
    lib.sdf_last_error.argtypes = []
    fp = ctypes.POINTER(ctypes.c_float)
    lib.sdf_query_rigid.restype = ctypes.c_int
    lib.sdf_query_rigid.argtypes = [vp, fp, vp, i64, vp, vp]
    lib.sdf_query_grad_rigid.restype = ctypes.c_int
    lib.sdf_query_grad_rigid.argtypes = [vp, fp, vp, i64, vp, vp, vp]
    lib.collide_project_rigid.restype = ctypes.c_int
    lib.collide_project_rigid.argtypes = [vp, fp, vp, i64, f32, vp, vp, vp, vp]
    lib.sdf_group_create.restype = ctypes.c_int
    lib.sdf_group_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int, ctypes.POINTER(vp),
                                     ctypes.POINTER(i64), f32, ctypes.POINTER(vp)]
    lib.sdf_group_collide_project.restype = ctypes.c_int
    lib.sdf_group_collide_project.argtypes = [vp, vp]
    lib.sdf_net_autotune.restype = ctypes.c_int
    lib.sdf_net_autotune.argtypes = [vp, i64, vp, ctypes.POINTER(ctypes.c_int)]
    lib.sdf_net_set_tile_variant.restype = ctypes.c_int
    lib.sdf_net_set_tile_variant.argtypes = [vp, ctypes.c_int]
    lib.sdf_group_set_launch.restype = ctypes.c_int
    lib.sdf_group_set_launch.argtypes = [vp, ctypes.c_int]
    lib.sdf_group_autotune.restype = ctypes.c_int
    lib.sdf_group_autotune.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_int)]
    lib.sdf_verlet_step.restype = ctypes.c_int
    lib.sdf_verlet_step.argtypes = [vp, vp, i64, f32, ctypes.POINTER(ctypes.c_float), f32, vp]
    lib.sdf_group_destroy.restype = ctypes.c_int
    lib.sdf_group_destroy.argtypes = [vp]
    lib.sdf_train_workspace_bytes.restype = i64
    lib.sdf_train_workspace_bytes.argtypes = [desc_p, i64]
    lib.sdf_train_step.restype = ctypes.c_int
    lib.sdf_train_step.argtypes = [desc_p, vp, vp, vp, i64, f32, vp, vp, vp, ctypes.c_size_t, vp]
    lib.sdf_train_step_noalloc.restype = ctypes.c_int
    lib.sdf_train_step_noalloc.argtypes = [desc_p, vp, vp, vp, i64, f32, vp, vp, vp]
    return lib


lib = _load()


def sdf_last_error() -> str:
    return lib.sdf_last_error().decode()


def _check(rc):
    if rc != SDF_OK:
        raise SdfError(rc, sdf_last_error())
    return rc


def make_desc(widths, skip=0, beta=100.0, precision="fp32", fourier=0) -> sdf_net_desc:
    d = sdf_net_desc()
    d.n_hidden = len(widths)
    for i, w in enumerate(widths):
        d.width[i] = int(w)
    d.skip_layer = int(skip)
    d.beta = float(beta)
    d.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    d.fourier = int(fourier)
    return d


def sdf_param_count(desc: sdf_net_desc) -> int:
    return int(lib.sdf_param_count(ctypes.byref(desc)))


def sdf_net_create(desc: sdf_net_desc, params_host, device: int = 0):
    """params_host: contiguous float32 numpy array (host).  Returns a handle (int)."""
    import numpy as np
    p = np.ascontiguousarray(params_host, dtype=np.float32)
    h = ctypes.c_void_p()
    _check(lib.sdf_net_create(ctypes.byref(desc), p.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                              p.size, int(device), ctypes.byref(h)))
    return h.value


def sdf_net_destroy(handle):
    return _check(lib.sdf_net_destroy(handle))


def _ptr(t):
    return None if t is None else t.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return int(stream)


def sdf_query(handle, pts, n, sdf, stream=None):
    return _check(lib.sdf_query(handle, _ptr(pts), int(n), _ptr(sdf), _stream(stream)))


def sdf_query_grad(handle, pts, n, sdf, grad, stream=None):
    return _check(lib.sdf_query_grad(handle, _ptr(pts), int(n), _ptr(sdf), _ptr(grad), _stream(stream)))


def collide_project(handle, pts, n, eps, sdf=None, normal=None, hit=None, stream=None):
    return _check(lib.collide_project(handle, _ptr(pts), int(n), float(eps), _ptr(sdf), _ptr(normal),
                                      _ptr(hit), _stream(stream)))


class SdfNet:
    """Owner of one packed network on one device; methods take torch CUDA tensors."""

    def __init__(self, spec, params, precision="fp32", device=0):
        self.spec = spec
        self.precision = precision
        self.device = device
        self.desc = make_desc(spec.widths, spec.skip, spec.beta, precision, getattr(spec, "fourier", 0))
        self.handle = sdf_net_create(self.desc, params, device)

    def autotune(self, n_sample=1 << 18, stream=None) -> int:
        """Time the collide_project tile variants and keep the faster; returns its index."""
        return sdf_net_autotune(self.handle, n_sample, stream)

    def set_tile_variant(self, variant: int):
        _check(lib.sdf_net_set_tile_variant(self.handle, int(variant)))

    def close(self):
        if self.handle:
            sdf_net_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _pts(pts):
        import torch
        if not (pts.is_cuda and pts.dtype == torch.float32 and pts.is_contiguous()
                and pts.dim() == 2 and pts.shape[1] == 3):
            raise ValueError("pts must be a contiguous float32 CUDA tensor of shape [n, 3]")
        return pts

    def query(self, pts, out=None, T=None):
        """f at every point; T (4x4, optional): the network's frame in the world."""
        import torch
        pts = self._pts(pts)
        out = torch.empty(pts.shape[0], device=pts.device, dtype=torch.float32) if out is None else out
        if T is None:
            sdf_query(self.handle, pts, pts.shape[0], out)
        else:
            sdf_query_rigid(self.handle, T, pts, pts.shape[0], out)
        return out

    def query_grad(self, pts, sdf=None, grad=None, T=None):
        import torch
        pts = self._pts(pts)
        n = pts.shape[0]
        sdf = torch.empty(n, device=pts.device, dtype=torch.float32) if sdf is None else sdf
        grad = torch.empty(n, 3, device=pts.device, dtype=torch.float32) if grad is None else grad
        if T is None:
            sdf_query_grad(self.handle, pts, n, sdf, grad)
        else:
            sdf_query_grad_rigid(self.handle, T, pts, n, sdf, grad)
        return sdf, grad

    def collide_project(self, pts, eps, want=("sdf", "normal", "hit"), T=None):
        """In place on pts; returns the requested optional outputs."""
        import torch
        pts = self._pts(pts)
        n = pts.shape[0]
        outs = {}
        if "sdf" in want:
            outs["sdf"] = torch.empty(n, device=pts.device, dtype=torch.float32)
        if "normal" in want:
            outs["normal"] = torch.empty(n, 3, device=pts.device, dtype=torch.float32)
        if "hit" in want:
            outs["hit"] = torch.empty(n, device=pts.device, dtype=torch.uint8)
        if T is None:
            collide_project(self.handle, pts, n, eps, outs.get("sdf"), outs.get("normal"), outs.get("hit"))
        else:
            collide_project_rigid(self.handle, T, pts, n, eps, outs.get("sdf"), outs.get("normal"),
                                  outs.get("hit"))
        return outs


def _frame(T):
    import numpy as np
    t = np.ascontiguousarray(T, dtype=np.float32).reshape(16)
    return t, t.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def sdf_query_rigid(handle, T, pts, n, sdf, stream=None):
    t, tp = _frame(T)
    return _check(lib.sdf_query_rigid(handle, tp, _ptr(pts), int(n), _ptr(sdf), _stream(stream)))


def sdf_query_grad_rigid(handle, T, pts, n, sdf, grad, stream=None):
    t, tp = _frame(T)
    return _check(lib.sdf_query_grad_rigid(handle, tp, _ptr(pts), int(n), _ptr(sdf), _ptr(grad),
                                           _stream(stream)))


def collide_project_rigid(handle, T, pts, n, eps, sdf=None, normal=None, hit=None, stream=None):
    t, tp = _frame(T)
    return _check(lib.collide_project_rigid(handle, tp, _ptr(pts), int(n), float(eps), _ptr(sdf),
                                            _ptr(normal), _ptr(hit), _stream(stream)))


# ------------------------------------------------------------------ fitting

def sdf_train_workspace_bytes(desc: sdf_net_desc, n: int) -> int:
    v = int(lib.sdf_train_workspace_bytes(ctypes.byref(desc), int(n)))
    if v < 0:
        raise SdfError(SDF_EINVAL, sdf_last_error())
    return v


def sdf_train_step(desc, params, pts, target, n, delta, grad_params, loss, workspace, ws_bytes,
                   stream=None):
    return _check(lib.sdf_train_step(ctypes.byref(desc), _ptr(params), _ptr(pts), _ptr(target), int(n),
                                     float(delta), _ptr(grad_params), _ptr(loss), _ptr(workspace),
                                     int(ws_bytes), _stream(stream)))


def sdf_train_step_noalloc(desc, params, pts, target, n, delta, grad_params, loss, stream=None):
    """sdf_train_step with the library's static scratch: no workspace, no allocation."""
    return _check(lib.sdf_train_step_noalloc(ctypes.byref(desc), _ptr(params), _ptr(pts), _ptr(target),
                                             int(n), float(delta), _ptr(grad_params), _ptr(loss),
                                             _stream(stream)))


class SdfFit:
    """Owns the device workspace of FP32 fitting steps for one network shape."""

    def __init__(self, spec, max_n, device=0):
        import torch
        self.spec = spec
        self.desc = make_desc(spec.widths, spec.skip, spec.beta, "fp32")
        self.device = torch.device("cuda", device)
        with torch.cuda.device(self.device):
            self.ws_bytes = sdf_train_workspace_bytes(self.desc, max_n)
        self.max_n = max_n
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)

    def step(self, params, pts, target, delta=0.1):
        """(loss, grad) for flat float32 CUDA parameters; both are new tensors."""
        import torch
        n = pts.shape[0]
        if n > self.max_n:
            raise ValueError("batch larger than the workspace was sized for")
        for t, shape in ((params, None), (pts, (n, 3)), (target, (n,))):
            if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
                raise ValueError("params, pts and target must be contiguous float32 CUDA tensors")
            if shape is not None and tuple(t.shape) != shape:
                raise ValueError("pts must be [n, 3] and target [n]")
        grad = torch.empty_like(params)
        loss = torch.empty(1, device=params.device, dtype=torch.float32)
        sdf_train_step(self.desc, params, pts, target, n, delta, grad, loss, self.workspace, self.ws_bytes)
        return loss, grad


def fit_loss(fit: SdfFit, params, pts, target, delta=0.1):
    """Differentiable clamped-L1 fitting loss: the gradient w.r.t. params comes
    from the library's reverse sweep and weight-gradient kernels."""
    import torch

    class _FitLoss(torch.autograd.Function):
        @staticmethod
        def forward(ctx, p):
            loss, grad = fit.step(p.detach().contiguous(), pts, target, delta)
            ctx.save_for_backward(grad)
            return loss[0]

        @staticmethod
        def backward(ctx, gout):
            (grad,) = ctx.saved_tensors
            return gout * grad

    return _FitLoss.apply(params)


# ------------------------------------------------------------ grouped calls

def sdf_group_create(handles, pts_ptrs, counts, eps):
    n = len(handles)
    H = (ctypes.c_void_p * n)(*handles)
    P = (ctypes.c_void_p * n)(*pts_ptrs)
    C = (ctypes.c_int64 * n)(*counts)
    g = ctypes.c_void_p()
    _check(lib.sdf_group_create(H, n, P, C, float(eps), ctypes.byref(g)))
    return g.value


def sdf_group_collide_project(group, stream=None):
    return _check(lib.sdf_group_collide_project(group, _stream(stream)))


def sdf_group_destroy(group):
    return _check(lib.sdf_group_destroy(group))


def sdf_net_autotune(handle, n_sample=1 << 18, stream=None) -> int:
    v = ctypes.c_int(0)
    _check(lib.sdf_net_autotune(handle, int(n_sample), _stream(stream), ctypes.byref(v)))
    return v.value


def sdf_group_autotune(group, stream=None) -> int:
    """Times the launch modes and keeps the fastest; returns its SDF_GROUP_* value."""
    v = ctypes.c_int(0)
    _check(lib.sdf_group_autotune(group, _stream(stream), ctypes.byref(v)))
    return v.value


def sdf_group_set_launch(group, mode):
    return _check(lib.sdf_group_set_launch(group, GROUP_MODES.get(mode, mode)))


def verlet_step(pts, prev, dt, gravity=(0.0, 0.0, -9.81), damping=0.0, stream=None):
    """One explicit-Verlet step of the vertex tensors (in place; both [n, 3] float32 CUDA)."""
    import numpy as np
    g = np.ascontiguousarray(gravity, dtype=np.float32).reshape(3)
    SdfNet._pts(pts)
    SdfNet._pts(prev)
    if pts.shape != prev.shape:
        raise ValueError("pts and prev must have the same shape")
    _check(lib.sdf_verlet_step(_ptr(pts), _ptr(prev), pts.shape[0], float(dt),
                               g.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), float(damping), _stream(stream)))


class SdfGroup:
    """A fixed set of (network, vertex tensor) pairs projected in one pass."""

    def __init__(self, nets, pts_list, eps):
        for p in pts_list:
            SdfNet._pts(p)
        self.nets, self.pts = list(nets), list(pts_list)
        self.handle = sdf_group_create([n.handle for n in self.nets], [p.data_ptr() for p in self.pts],
                                       [p.shape[0] for p in self.pts], eps)

    def collide_project(self, stream=None):
        sdf_group_collide_project(self.handle, stream)

    def autotune(self, stream=None) -> int:
        """Pick tile variants and the launch mode by timing; returns the SDF_GROUP_* mode."""
        return sdf_group_autotune(self.handle, stream)

    def set_launch(self, mode):
        """"per_width", "per_network" or "persistent" (or an SDF_GROUP_* value)."""
        sdf_group_set_launch(self.handle, mode)

    def close(self):
        if self.handle:
            sdf_group_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
