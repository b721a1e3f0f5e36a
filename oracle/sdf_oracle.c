/*
 * sdf_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, FP64 CPU reference for neural-implicit-surface collision
 * handling (Bertiche, Madadi, Escalera, arXiv 2110.01614).  Only the tests,
 * the package's smoke check and the benchmark's CPU-baseline leg may load this
 * library.  It shares no code, header, table or constant with the HIP path.
 *
 * What it computes, each function citing the passage it follows:
 *   orc_mlp_eval     f(p) (Sec. 3.1, Eq. 1) and its input gradient by reverse
 *                    mode ("back-propagation", Sec. 3.2 after Eq. 3).
 *   orc_mlp_jvp      the same gradient by forward mode (a second algorithm for
 *                    the same quantity, used to pin the first).
 *   orc_collide      normal N = grad f / |grad f| (Eq. 2), detection f < eps
 *                    (Sec. 3.2) and the move to the contact point (Eq. 3).
 *   orc_point_tri    closest-point distance from a point to a triangle by
 *                    Voronoi-region classification (Ericson, cited in Sec. 1-2).
 *   orc_mesh_sdf     brute-force vertex-triangle signed distance (Sec. 1-2's
 *                    naive approach; sign from the generalised winding number,
 *                    interior negative as in Sec. 3.2).
 *   orc_fit_loss     clamped-L1 fitting loss and its parameter gradient
 *                    (Sec. 3.1 L1 loss, clamped as the fitting workload states).
 *
 * Network convention (parameters read as float32, widened to double): L hidden
 * layers, h_0 = x, u_l = [h_{l-1}; x] at the skip layer else h_{l-1},
 * z_l = W_l u_l + b_l, h_l = softplus_beta(z_l), f = w_o . h_L + b_o.
 * softplus_beta(z) = max(z,0) + log1p(exp(-beta|z|))/beta; its derivative is
 * sigmoid(beta z).  Flat layout: per hidden layer W_l row-major [w_l][K_l] then
 * b_l, then w_o[w_L], b_o.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static int nthreads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

static int thread_id(void) {
#ifdef _OPENMP
  return omp_get_thread_num();
#else
  return 0;
#endif
}

#define ORC_MAXL 32
#define ORC_PI 3.14159265358979323846

typedef struct {
  int L;
  int w[ORC_MAXL];
  int skip;
  double beta;
} net_t;

static int net_init(net_t* n, int L, const int* widths, int skip, double beta) {
  if (L < 1 || L > ORC_MAXL) return -1;
  if (skip == 1 || skip < 0 || skip > L) return -1;
  n->L = L;
  n->skip = skip;
  n->beta = beta;
  for (int i = 0; i < L; ++i) {
    if (widths[i] < 1) return -1;
    n->w[i] = widths[i];
  }
  return 0;
}

/* K_l: inputs of hidden layer l (1-based). */
static int k_in(const net_t* n, int l) {
  int k = (l == 1) ? 3 : n->w[l - 2];
  return k + ((l == n->skip) ? 3 : 0);
}

static int max_width(const net_t* n) {
  int m = 3;
  for (int i = 0; i < n->L; ++i) m = n->w[i] > m ? n->w[i] : m;
  return m;
}

int64_t orc_param_count(int L, const int* widths, int skip) {
  net_t n;
  if (net_init(&n, L, widths, skip, 1.0)) return -1;
  int64_t c = 0;
  for (int l = 1; l <= L; ++l) c += (int64_t)n.w[l - 1] * k_in(&n, l) + n.w[l - 1];
  return c + n.w[L - 1] + 1;
}

static double softplus(double z, double beta) {
  return fmax(z, 0.0) + log1p(exp(-beta * fabs(z))) / beta;
}

static double sigmoid(double z, double beta) {
  double a = beta * z;
  if (a >= 0.0) return 1.0 / (1.0 + exp(-a));
  double e = exp(a);
  return e / (1.0 + e);
}

/* Offsets of W_l, b_l (l = 1..L) and of w_o, b_o inside the flat array. */
static void layer_offsets(const net_t* n, int64_t* offW, int64_t* offb, int64_t* offo) {
  int64_t o = 0;
  for (int l = 1; l <= n->L; ++l) {
    offW[l] = o;
    o += (int64_t)n->w[l - 1] * k_in(n, l);
    offb[l] = o;
    o += n->w[l - 1];
  }
  *offo = o;
}

/*
 * Forward pass for one point; keeps z_l (pre-activations) and h_l for every
 * layer in zs/hs ([L][maxw]).  Returns f.
 */
static double forward_point(const net_t* n, const double* P, const int64_t* offW,
                            const int64_t* offb, int64_t offo, const double* x,
                            double* zs, double* hs, int ld) {
  const double* prev = x;
  int prev_n = 3;
  for (int l = 1; l <= n->L; ++l) {
    const int out = n->w[l - 1], K = k_in(n, l);
    const double* W = P + offW[l];
    const double* b = P + offb[l];
    double* z = zs + (int64_t)(l - 1) * ld;
    double* h = hs + (int64_t)(l - 1) * ld;
    for (int j = 0; j < out; ++j) {
      const double* row = W + (int64_t)j * K;
      double s = b[j];
      for (int k = 0; k < prev_n; ++k) s += row[k] * prev[k];
      if (l == n->skip)
        for (int c = 0; c < 3; ++c) s += row[prev_n + c] * x[c];
      z[j] = s;
      h[j] = softplus(s, n->beta);
    }
    prev = h;
    prev_n = out;
  }
  const double* wo = P + offo;
  double f = wo[prev_n];
  for (int j = 0; j < prev_n; ++j) f += wo[j] * prev[j];
  return f;
}

/*
 * Reverse mode: d_L = w_o (.) sigma(beta z_L); g_l = W_l^T d_l; the skip
 * columns of g_l go to grad x; d_{l-1} = g_l[:w_{l-1}] (.) sigma(beta z_{l-1});
 * layer 1's g is the rest of grad x.
 */
static void reverse_point(const net_t* n, const double* P, const int64_t* offW,
                          int64_t offo, const double* zs, int ld, double* d, double* dn,
                          double* gx) {
  const double* wo = P + offo;
  const int WL = n->w[n->L - 1];
  const double* zL = zs + (int64_t)(n->L - 1) * ld;
  for (int j = 0; j < WL; ++j) d[j] = wo[j] * sigmoid(zL[j], n->beta);
  gx[0] = gx[1] = gx[2] = 0.0;
  for (int l = n->L; l >= 1; --l) {
    const int out = n->w[l - 1], K = k_in(n, l);
    const int prev_n = (l == 1) ? 3 : n->w[l - 2];
    const double* W = P + offW[l];
    for (int k = 0; k < K; ++k) {
      double s = 0.0;
      for (int j = 0; j < out; ++j) s += W[(int64_t)j * K + k] * d[j];
      if (k >= prev_n) {
        gx[k - prev_n] += s; /* skip columns */
      } else if (l == 1) {
        gx[k] += s;
      } else {
        dn[k] = s * sigmoid(zs[(int64_t)(l - 2) * ld + k], n->beta);
      }
    }
    if (l > 1) memcpy(d, dn, sizeof(double) * prev_n);
  }
}

int orc_mlp_eval(int L, const int* widths, int skip, double beta, const double* P,
                 int64_t npts, const double* X, double* f, double* grad) {
  net_t n;
  if (net_init(&n, L, widths, skip, beta)) return -1;
  int64_t offW[ORC_MAXL + 1], offb[ORC_MAXL + 1], offo;
  layer_offsets(&n, offW, offb, &offo);
  const int ld = max_width(&n);
  const size_t per = (size_t)L * ld * 2 + 2 * (size_t)ld;
  double* pool = (double*)malloc(sizeof(double) * per * (size_t)nthreads());
  if (!pool) return -2;
#pragma omp parallel
  {
    double* zs = pool + per * (size_t)thread_id();
    double* hs = zs + (size_t)L * ld;
    double* d = hs + (size_t)L * ld;
    double* dn = d + ld;
#pragma omp for schedule(static)
    for (int64_t i = 0; i < npts; ++i) {
      const double* x = X + 3 * i;
      double fi = forward_point(&n, P, offW, offb, offo, x, zs, hs, ld);
      if (f) f[i] = fi;
      if (grad) reverse_point(&n, P, offW, offo, zs, ld, d, dn, grad + 3 * i);
    }
  }
  free(pool);
  return 0;
}

/*
 * Forward mode: J_0 = I; J_l = diag(sigma(beta z_l)) (W_l [J_{l-1}; I_skip]);
 * grad f = w_o^T J_L.  A different algorithm for the same gradient.
 */
int orc_mlp_jvp(int L, const int* widths, int skip, double beta, const double* P,
                int64_t npts, const double* X, double* f, double* grad) {
  net_t n;
  if (net_init(&n, L, widths, skip, beta)) return -1;
  int64_t offW[ORC_MAXL + 1], offb[ORC_MAXL + 1], offo;
  layer_offsets(&n, offW, offb, &offo);
  const int ld = max_width(&n);
  const size_t per = 8 * (size_t)ld;
  double* pool = (double*)malloc(sizeof(double) * per * (size_t)nthreads());
  if (!pool) return -2;
#pragma omp parallel
  {
    {
      double* buf = pool + per * (size_t)thread_id();
      double* h = buf;
      double* hn = h + ld;
      double* J = hn + ld;     /* [ld][3] */
      double* Jn = J + 3 * ld; /* [ld][3] */
#pragma omp for schedule(static)
      for (int64_t i = 0; i < npts; ++i) {
        const double* x = X + 3 * i;
        int prev_n = 3;
        for (int k = 0; k < 3; ++k) {
          h[k] = x[k];
          for (int c = 0; c < 3; ++c) J[3 * k + c] = (k == c) ? 1.0 : 0.0;
        }
        for (int l = 1; l <= L; ++l) {
          const int out = n.w[l - 1], K = k_in(&n, l);
          const double* W = P + offW[l];
          const double* b = P + offb[l];
          for (int j = 0; j < out; ++j) {
            const double* row = W + (int64_t)j * K;
            double z = b[j], t0 = 0.0, t1 = 0.0, t2 = 0.0;
            for (int k = 0; k < prev_n; ++k) {
              z += row[k] * h[k];
              t0 += row[k] * J[3 * k];
              t1 += row[k] * J[3 * k + 1];
              t2 += row[k] * J[3 * k + 2];
            }
            if (l == n.skip) {
              for (int c = 0; c < 3; ++c) z += row[prev_n + c] * x[c];
              t0 += row[prev_n];
              t1 += row[prev_n + 1];
              t2 += row[prev_n + 2];
            }
            const double s = sigmoid(z, beta);
            hn[j] = softplus(z, beta);
            Jn[3 * j] = s * t0;
            Jn[3 * j + 1] = s * t1;
            Jn[3 * j + 2] = s * t2;
          }
          memcpy(h, hn, sizeof(double) * out);
          memcpy(J, Jn, sizeof(double) * 3 * out);
          prev_n = out;
        }
        const double* wo = P + offo;
        double fi = wo[prev_n], g0 = 0.0, g1 = 0.0, g2 = 0.0;
        for (int j = 0; j < prev_n; ++j) {
          fi += wo[j] * h[j];
          g0 += wo[j] * J[3 * j];
          g1 += wo[j] * J[3 * j + 1];
          g2 += wo[j] * J[3 * j + 2];
        }
        if (f) f[i] = fi;
        if (grad) {
          grad[3 * i] = g0;
          grad[3 * i + 1] = g1;
          grad[3 * i + 2] = g2;
        }
      }
    }
  }
  free(pool);
  return 0;
}

/*
 * Collision step for given f and grad f (Sec. 3.2): N = grad/|grad| (Eq. 2),
 * 0 when |grad| = 0; hit = f < eps (strict; NaN is no hit); a hit vertex with
 * nonzero normal moves to p + (eps - f) N, the contact-point offset of Eq. 3
 * applied to the vertex.  Any other vertex is copied unchanged.
 */
void orc_collide(int64_t npts, const double* Pin, const double* f, const double* grad,
                 double eps, double* Pout, double* normal, uint8_t* hit) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < npts; ++i) {
    const double* g = grad + 3 * i;
    const double nrm = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
    double N[3] = {0.0, 0.0, 0.0};
    if (nrm > 0.0)
      for (int c = 0; c < 3; ++c) N[c] = g[c] / nrm;
    const int h = f[i] < eps;
    for (int c = 0; c < 3; ++c) {
      double p = Pin[3 * i + c];
      if (h && nrm > 0.0) p = p + (eps - f[i]) * N[c];
      if (Pout) Pout[3 * i + c] = p;
      if (normal) normal[3 * i + c] = N[c];
    }
    if (hit) hit[i] = (uint8_t)h;
  }
}

/* ---------------------------------------------------------------- meshes */

static double dot3(const double* a, const double* b) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

/*
 * Squared distance from p to triangle (a,b,c) and the closest point q, by
 * classifying p into the Voronoi region of a vertex, an edge or the face.
 * Returns the region: 0,1,2 vertex a,b,c; 3 edge ab, 4 edge bc, 5 edge ca;
 * 6 face interior.
 */
int orc_point_tri(const double* p, const double* a, const double* b, const double* c,
                  double* q, double* dist2) {
  double ab[3], ac[3], ap[3], bp[3], cp[3];
  for (int k = 0; k < 3; ++k) {
    ab[k] = b[k] - a[k];
    ac[k] = c[k] - a[k];
    ap[k] = p[k] - a[k];
    bp[k] = p[k] - b[k];
    cp[k] = p[k] - c[k];
  }
  int region;
  double s = 0.0, t = 0.0; /* q = a + s ab + t ac */
  const double d1 = dot3(ab, ap), d2 = dot3(ac, ap);
  const double d3 = dot3(ab, bp), d4 = dot3(ac, bp);
  const double d5 = dot3(ab, cp), d6 = dot3(ac, cp);
  const double vc = d1 * d4 - d3 * d2;
  const double vb = d5 * d2 - d1 * d6;
  const double va = d3 * d6 - d5 * d4;
  if (d1 <= 0.0 && d2 <= 0.0) {
    region = 0;
  } else if (d3 >= 0.0 && d4 <= d3) {
    region = 1;
    s = 1.0;
  } else if (d6 >= 0.0 && d5 <= d6) {
    region = 2;
    t = 1.0;
  } else if (vc <= 0.0 && d1 >= 0.0 && d3 <= 0.0) {
    region = 3;
    s = d1 / (d1 - d3);
  } else if (va <= 0.0 && (d4 - d3) >= 0.0 && (d5 - d6) >= 0.0) {
    region = 4;
    const double w = (d4 - d3) / ((d4 - d3) + (d5 - d6));
    s = 1.0 - w;
    t = w;
  } else if (vb <= 0.0 && d2 >= 0.0 && d6 <= 0.0) {
    region = 5;
    t = d2 / (d2 - d6);
  } else {
    region = 6;
    const double den = 1.0 / (va + vb + vc);
    s = vb * den;
    t = vc * den;
  }
  double qq[3], dd = 0.0;
  for (int k = 0; k < 3; ++k) {
    qq[k] = a[k] + s * ab[k] + t * ac[k];
    const double e = p[k] - qq[k];
    dd += e * e;
  }
  if (q) memcpy(q, qq, sizeof qq);
  if (dist2) *dist2 = dd;
  return region;
}

/* Signed solid angle of triangle (a,b,c) seen from p (Van Oosterom & Strackee). */
double orc_solid_angle(const double* p, const double* A, const double* B, const double* C) {
  double a[3], b[3], c[3];
  for (int k = 0; k < 3; ++k) {
    a[k] = A[k] - p[k];
    b[k] = B[k] - p[k];
    c[k] = C[k] - p[k];
  }
  const double la = sqrt(dot3(a, a)), lb = sqrt(dot3(b, b)), lc = sqrt(dot3(c, c));
  const double det = a[0] * (b[1] * c[2] - b[2] * c[1]) - a[1] * (b[0] * c[2] - b[2] * c[0]) +
                     a[2] * (b[0] * c[1] - b[1] * c[0]);
  const double den = la * lb * lc + dot3(a, b) * lc + dot3(b, c) * la + dot3(c, a) * lb;
  return 2.0 * atan2(det, den);
}

/*
 * Brute force over every (point, triangle) pair: unsigned distance is the
 * minimum closest-point distance; the sign is negative where the generalised
 * winding number sum(Omega_t)/(4 pi) exceeds 1/2 (inside).  Also returns the
 * winding numbers when wind != NULL.
 */
void orc_mesh_sdf(int64_t nv, const double* V, int64_t nt, const int32_t* T, int64_t npts,
                  const double* X, double* sdf, double* wind) {
  (void)nv;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = 0; i < npts; ++i) {
    const double* p = X + 3 * i;
    double best = INFINITY, omega = 0.0;
    for (int64_t t = 0; t < nt; ++t) {
      const double* a = V + 3 * (int64_t)T[3 * t];
      const double* b = V + 3 * (int64_t)T[3 * t + 1];
      const double* c = V + 3 * (int64_t)T[3 * t + 2];
      double d2;
      orc_point_tri(p, a, b, c, NULL, &d2);
      if (d2 < best) best = d2;
      omega += orc_solid_angle(p, a, b, c);
    }
    const double w = omega / (4.0 * ORC_PI);
    if (wind) wind[i] = w;
    if (sdf) sdf[i] = (w > 0.5 ? -1.0 : 1.0) * sqrt(best);
  }
}

/* ------------------------------------------------------------ fitting */

/*
 * Clamped-L1 loss L = mean_i |clamp(f_i) - clamp(s_i)| (clamp to [-delta,
 * delta]) and dL/dparams by back-propagation through the network.
 * dL/df_i = sign(clamp(f_i) - clamp(s_i)) * [ -delta <= f_i <= delta ] / n,
 * sign(0) = 0.  grad (n_params doubles) is overwritten.  Returns L via *loss.
 */
int orc_fit_loss(int L, const int* widths, int skip, double beta, const double* P,
                 int64_t npts, const double* X, const double* S, double delta, double* loss,
                 double* grad) {
  net_t n;
  if (net_init(&n, L, widths, skip, beta)) return -1;
  int64_t offW[ORC_MAXL + 1], offb[ORC_MAXL + 1], offo;
  layer_offsets(&n, offW, offb, &offo);
  const int64_t np = orc_param_count(L, widths, skip);
  const int ld = max_width(&n);
  memset(grad, 0, sizeof(double) * (size_t)np);
  double total = 0.0;
  const size_t per = (size_t)L * ld * 2 + 2 * (size_t)ld;
  const int nt = nthreads();
  double* pool = (double*)malloc(sizeof(double) * per * (size_t)nt);
  double* gpool = (double*)calloc((size_t)np * (size_t)nt, sizeof(double));
  double* lpool = (double*)calloc((size_t)nt, sizeof(double));
  if (!pool || !gpool || !lpool) {
    free(pool);
    free(gpool);
    free(lpool);
    return -2;
  }
#pragma omp parallel
  {
    double* g = gpool + (size_t)np * (size_t)thread_id();
    double* zs = pool + per * (size_t)thread_id();
    double part = 0.0;
    {
      double* hs = zs + (size_t)L * ld;
      double* e = hs + (size_t)L * ld;
      double* en = e + ld;
#pragma omp for schedule(static)
      for (int64_t i = 0; i < npts; ++i) {
        const double* x = X + 3 * i;
        const double fi = forward_point(&n, P, offW, offb, offo, x, zs, hs, ld);
        const double cf = fmin(fmax(fi, -delta), delta);
        const double cs = fmin(fmax(S[i], -delta), delta);
        const double r = cf - cs;
        part += fabs(r);
        const double sg = (r > 0.0) - (r < 0.0);
        const double u = (fi >= -delta && fi <= delta) ? sg / (double)npts : 0.0;
        if (u == 0.0) continue;
        const int WL = n.w[L - 1];
        const double* hL = hs + (int64_t)(L - 1) * ld;
        const double* wo = P + offo;
        for (int j = 0; j < WL; ++j) {
          g[offo + j] += u * hL[j];
          e[j] = u * wo[j] * sigmoid(zs[(int64_t)(L - 1) * ld + j], beta);
        }
        g[offo + WL] += u;
        for (int l = L; l >= 1; --l) {
          const int out = n.w[l - 1], K = k_in(&n, l);
          const int prev_n = (l == 1) ? 3 : n.w[l - 2];
          const double* hprev = (l == 1) ? x : hs + (int64_t)(l - 2) * ld;
          const double* W = P + offW[l];
          double* gW = g + offW[l];
          double* gb = g + offb[l];
          for (int j = 0; j < out; ++j) {
            const double ej = e[j];
            double* row = gW + (int64_t)j * K;
            for (int k = 0; k < prev_n; ++k) row[k] += ej * hprev[k];
            if (l == skip)
              for (int c = 0; c < 3; ++c) row[prev_n + c] += ej * x[c];
            gb[j] += ej;
          }
          if (l > 1) {
            for (int k = 0; k < prev_n; ++k) {
              double s = 0.0;
              for (int j = 0; j < out; ++j) s += W[(int64_t)j * K + k] * e[j];
              en[k] = s * sigmoid(zs[(int64_t)(l - 2) * ld + k], beta);
            }
            memcpy(e, en, sizeof(double) * prev_n);
          }
        }
      }
      lpool[thread_id()] = part;
    }
  }
  /* fixed-order reduction of the per-thread losses and gradients */
  for (int t = 0; t < nt; ++t) {
    total += lpool[t];
    for (int64_t k = 0; k < np; ++k) grad[k] += gpool[(size_t)np * t + k];
  }
  free(pool);
  free(gpool);
  free(lpool);
  if (loss) *loss = total / (double)(npts > 0 ? npts : 1);
  return 0;
}
