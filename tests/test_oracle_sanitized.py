"""The FP64 oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(gcc, host code only) and driven through every entry point, including its
error paths and degenerate inputs.  Any out-of-bounds access, leak, signed
overflow or other undefined behaviour aborts the test program."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "sdf_oracle.c")

DRIVER = r"""
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
int64_t orc_param_count(int L, const int* widths, int skip);
int orc_mlp_eval(int L, const int* widths, int skip, double beta, const double* P, int64_t npts,
                 const double* X, double* f, double* grad);
int orc_mlp_jvp(int L, const int* widths, int skip, double beta, const double* P, int64_t npts,
                const double* X, double* f, double* grad);
void orc_collide(int64_t npts, const double* Pin, const double* f, const double* grad, double eps,
                 double* Pout, double* normal, uint8_t* hit);
int orc_point_tri(const double* p, const double* a, const double* b, const double* c, double* q,
                  double* dist2);
double orc_solid_angle(const double* p, const double* A, const double* B, const double* C);
void orc_mesh_sdf(int64_t nv, const double* V, int64_t nt, const int32_t* T, int64_t npts,
                  const double* X, double* sdf, double* wind);
int orc_fit_loss(int L, const int* widths, int skip, double beta, const double* P, int64_t npts,
                 const double* X, const double* S, double delta, double* loss, double* grad);

static double rnd(unsigned* s) { *s = *s * 1664525u + 1013904223u; return (double)(*s >> 8) / 16777216.0 - 0.5; }

int main(void) {
  unsigned seed = 1;
  const int shapes[3][4] = {{3, 16, 0, 0}, {4, 8, 3, 0}, {2, 5, 2, 0}};
  for (int s = 0; s < 3; ++s) {
    int L = shapes[s][0], w = shapes[s][1], skip = shapes[s][2];
    int widths[8];
    for (int i = 0; i < L; ++i) widths[i] = w + i % 2;
    int64_t np = orc_param_count(L, widths, skip);
    if (np <= 0) return 10;
    double* P = malloc(sizeof(double) * np);
    for (int64_t i = 0; i < np; ++i) P[i] = rnd(&seed);
    const int64_t n = 37;
    double *X = malloc(sizeof(double) * 3 * n), *f = malloc(sizeof(double) * n), *g = malloc(sizeof(double) * 3 * n);
    double *f2 = malloc(sizeof(double) * n), *g2 = malloc(sizeof(double) * 3 * n), *S = malloc(sizeof(double) * n);
    for (int64_t i = 0; i < 3 * n; ++i) X[i] = 2.0 * rnd(&seed);
    for (int64_t i = 0; i < n; ++i) S[i] = rnd(&seed);
    if (orc_mlp_eval(L, widths, skip, 100.0, P, n, X, f, g)) return 11;
    if (orc_mlp_eval(L, widths, skip, 100.0, P, n, X, f2, NULL)) return 12;
    if (orc_mlp_jvp(L, widths, skip, 100.0, P, n, X, f2, g2)) return 13;
    for (int64_t i = 0; i < 3 * n; ++i) if (fabs(g[i] - g2[i]) > 1e-9 * (1 + fabs(g[i]))) return 14;
    double loss, *G = malloc(sizeof(double) * np);
    if (orc_fit_loss(L, widths, skip, 100.0, P, n, X, S, 0.1, &loss, G)) return 15;
    double *Po = malloc(sizeof(double) * 3 * n), *N = malloc(sizeof(double) * 3 * n);
    uint8_t* hit = malloc(n);
    f[0] = NAN;
    g[3] = g[4] = g[5] = 0.0;
    orc_collide(n, X, f, g, 0.005, Po, N, hit);
    free(P); free(X); free(f); free(g); free(f2); free(g2); free(S); free(G); free(Po); free(N); free(hit);
  }
  int bad[2] = {8, 8};
  if (orc_param_count(0, bad, 0) >= 0 && orc_param_count(2, bad, 1) >= 0) return 20;
  /* a tetrahedron: distances and winding numbers at inside, outside and on-vertex points */
  const double V[12] = {0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0, 1};
  const int32_t T[12] = {0, 2, 1, 0, 1, 3, 0, 3, 2, 1, 2, 3};
  const double Q[12] = {0.1, 0.1, 0.1, 2, 2, 2, 0, 0, 0, -1, 0.5, 0.5};
  double sd[4], wd[4], q[3], d2;
  orc_mesh_sdf(4, V, 4, T, 4, Q, sd, wd);
  if (!(sd[0] < 0 && sd[1] > 0)) return 21;
  orc_point_tri(Q, V, V + 3, V + 6, q, &d2);
  orc_point_tri(Q, V, V, V, q, &d2); /* degenerate triangle */
  (void)orc_solid_angle(V, V, V + 3, V + 6);
  printf("sanitized oracle ok\n");
  return 0;
}
"""


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    drv = tmp_path / "driver.c"
    drv.write_text(DRIVER)
    exe = tmp_path / "oracle_san"
    cmd = ["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", str(drv), SRC, "-o", str(exe), "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr, r.stderr
    assert "sanitized oracle ok" in r.stdout
