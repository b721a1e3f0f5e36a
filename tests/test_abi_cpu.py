"""Host-only checks of the C-ABI library: it loads into the same HIP runtime
as torch, exports every declared symbol, and rejects malformed arguments
before any kernel launch.  No test here needs a GPU."""
import ctypes
import os
import re
import subprocess
import sys

import numpy as np
import pytest

from paper_2110_01614_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sdfcollide.h")

B = pytest.importorskip("paper_2110_01614_amd.binding")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[\w]+\s*\*?\s*(\w+)\s*\(", text, flags=re.M)) -
                  {"if", "while"})


def test_one_hip_runtime_whatever_the_import_order():
    """Importing the binding before torch must not map a second HIP runtime
    (torch's bundled copy beside the system one): the runtime initialised
    second would see no device and every call would fail."""
    code = ("import paper_2110_01614_amd.binding as B, torch\n"
            "import ctypes\n"
            "ctypes.CDLL(B.LIB_PATH)\n"
            "r = B._hip_runtimes_mapped()\n"
            "assert len(r) == 1, r\n"
            "print('runtimes', sorted(r))\n")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True,
                         timeout=300)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "libamdhip64" in out.stdout


def test_library_exports_every_declared_function():
    names = declared_functions()
    assert {"sdf_query", "sdf_query_grad", "collide_project", "sdf_net_create"} <= set(names)
    lib = ctypes.CDLL(B.LIB_PATH)
    for name in names:
        assert hasattr(lib, name), name


@pytest.mark.parametrize("widths,skip", [((64, 64, 64), 0), ((256,) * 8, 5), ((128,) * 4, 2),
                                         ((7, 11, 5), 3)])
def test_param_count_matches_layout(widths, skip):
    spec = I.NetSpec(widths, skip)
    assert B.sdf_param_count(B.make_desc(widths, skip)) == I.param_count(spec)


@pytest.mark.parametrize("kw", [dict(widths=(64,), skip=1), dict(widths=(64, 64), skip=3),
                                dict(widths=(64, 0), skip=0), dict(widths=(64, 64), beta=float("nan")),
                                dict(widths=(64, 64), beta=-1.0), dict(widths=(64, 64), precision=9)])
def test_malformed_description_is_rejected(kw):
    d = B.make_desc(kw["widths"], kw.get("skip", 0), kw.get("beta", 100.0), kw.get("precision", 0))
    assert B.sdf_param_count(d) == -1
    with pytest.raises(B.SdfError) as e:
        B.sdf_net_create(d, np.zeros(16, np.float32))
    assert e.value.code == B.SDF_EINVAL


def test_param_count_mismatch_and_nonfinite_params():
    d = B.make_desc((64, 64, 64), 0)
    n = B.sdf_param_count(d)
    with pytest.raises(B.SdfError) as e:
        B.sdf_net_create(d, np.zeros(n - 1, np.float32))
    assert e.value.code == B.SDF_EINVAL
    p = np.zeros(n, np.float32)
    p[5] = np.inf
    with pytest.raises(B.SdfError) as e:
        B.sdf_net_create(d, p)
    assert e.value.code == B.SDF_EINVAL


@pytest.mark.parametrize("widths", [(96, 96), (64, 128), (512,) * 4, (64,) * 9, (64,)])
def test_unsupported_shapes_are_reported(widths):
    d = B.make_desc(widths, 0)
    with pytest.raises(B.SdfError) as e:
        B.sdf_net_create(d, np.zeros(B.sdf_param_count(d), np.float32))
    assert e.value.code == B.SDF_EUNSUPPORTED


@pytest.mark.parametrize("widths,precision", [((64,) * 4, "fp8"), ((96,) * 3, "fp8"), ((512,) * 3, "fp32")])
def test_precision_width_combinations_without_kernels(widths, precision):
    d = B.make_desc(widths, 0, precision=precision)
    with pytest.raises(B.SdfError) as e:
        B.sdf_net_create(d, np.zeros(B.sdf_param_count(d), np.float32))
    assert e.value.code == B.SDF_EUNSUPPORTED


def test_fourier_descriptions():
    from paper_2110_01614_amd import inputs as I
    spec = I.NetSpec((256,) * 4, fourier=128)
    d = B.make_desc(spec.widths, 0, precision="bf16", fourier=128)
    assert B.sdf_param_count(d) == I.param_count(spec)
    d = B.make_desc((256,) * 4, 2, precision="bf16", fourier=128)  # no skip with Fourier input
    assert B.sdf_param_count(d) == -1
    for widths, m, prec in [((256,) * 4, 64, "bf16"), ((256,) * 4, 128, "fp32"), ((256,) * 4, 128, "fp8")]:
        d = B.make_desc(widths, 0, precision=prec, fourier=m)
        with pytest.raises(B.SdfError) as e:
            B.sdf_net_create(d, np.zeros(B.sdf_param_count(d), np.float32))
        assert e.value.code == B.SDF_EUNSUPPORTED


def test_unknown_precision_is_rejected():
    d = B.make_desc((128,) * 3, 0)
    d.precision = 7
    assert B.sdf_param_count(d) == -1
    assert "precision" in B.sdf_last_error()


def test_null_handle_is_rejected_without_launch():
    assert B.lib.sdf_query(None, None, 5, None, None) == B.SDF_EINVAL
    assert "NULL" in B.sdf_last_error()
    assert B.lib.sdf_query_grad(None, None, 0, None, None, None) == B.SDF_EINVAL
    assert B.lib.collide_project(None, None, 0, 0.0, None, None, None, None) == B.SDF_EINVAL
    assert B.lib.sdf_net_destroy(None) == B.SDF_OK
