"""Plant plausible mistakes in a copy of the oracle (CPU only) and check that
the pin suite catches every one of them.  Nothing here touches a GPU."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "sdf_oracle.c")

MUTANTS = [
    ("softplus loses 1/beta", "log1p(exp(-beta * fabs(z))) / beta", "log1p(exp(-beta * fabs(z)))"),
    ("sigmoid sign flipped", "return 1.0 / (1.0 + exp(-a));", "return 1.0 / (1.0 + exp(a));"),
    ("skip columns dropped from grad", "gx[k - prev_n] += s; /* skip columns */", "(void)s;"),
    ("reverse uses the wrong layer's z", "dn[k] = s * sigmoid(zs[(int64_t)(l - 2) * ld + k]",
     "dn[k] = s * sigmoid(zs[(int64_t)(l - 1) * ld + k]"),
    ("skip fed h instead of x", "s += row[prev_n + c] * x[c];", "s += row[prev_n + c] * prev[c];"),
    ("projection moves the wrong way", "p = p + (eps - f[i]) * N[c];", "p = p + (f[i] - eps) * N[c];"),
    ("detection not strict", "const int h = f[i] < eps;", "const int h = f[i] <= eps;"),
    ("edge BC parameter swapped", "s = 1.0 - w;", "s = w;"),
    ("winding sign inverted", "(w > 0.5 ? -1.0 : 1.0)", "(w > 0.5 ? 1.0 : -1.0)"),
    ("solid angle term transposed", "dot3(b, c) * la", "dot3(b, c) * lb"),
    ("clamp mask ignored", "(fi >= -delta && fi <= delta) ? sg", "1 ? sg"),
    ("output bias dropped", "double f = wo[prev_n];", "double f = 0.0;"),
]


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_planted_mistake(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, "mutation site not unique: " + name
    path = tmp_path / "mutant.c"
    path.write_text(src.replace(old, new))
    lib = tmp_path / "libmutant.so"
    subprocess.check_call(["gcc", "-std=c11", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", str(lib),
                           str(path), "-lm"])
    env = dict(os.environ, SDF_ORACLE_LIB=str(lib), OMP_NUM_THREADS="4")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, "pins did not catch: " + name + "\n" + r.stdout[-2000:]
