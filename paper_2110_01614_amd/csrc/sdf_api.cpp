// sdf_api.cpp -- C ABI of the gfx950 neural-SDF collision library: argument
// checks, weight packing and kernel dispatch.  Declared in
// include/sdfcollide.h, which states the contract of every entry point.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <algorithm>
#include <cstring>
#include <string>
#include <mutex>
#include <vector>

#include "../../include/sdfcollide.h"
#include "sdf_device.hpp"

namespace sdfc {
template <int W, int PREC, int MODE, int VAR>
__global__ void sdf_k16(const KArgs a);
template <int W, int PREC, int MODE, int VAR>
__global__ void sdf_k16_group(const KArgs* nets, const int* tile_start, int n_nets, int tile0);
template <int PREC>
__global__ void sdf_k16_persist(const KArgs* nets, const int* width, const int* item_start, int n_nets, int* ctr);
template <int W, int MODE>
__global__ void sdf_k32(const KArgs a);
__global__ void pack_fp32_kernel(TrainNet t, const float* P, float* stream, float* small);
__global__ void verlet_kernel(float* x, float* xp, int64_t m, float k, float c0, float c1, float c2);
__global__ void fill_kernel(float* p, int64_t n, float v);
__global__ void loss_reduce_kernel(const float* terms, int64_t n, float* loss);
template <int BS>
__global__ void wgrad_kernel(TrainNet t, const float* E, const float* H, const float* U, int64_t n, int items,
                             int nsplit, float* part, float* grad);
template <int BS>
__global__ void wgrad_reduce_kernel(TrainNet t, const float* part, int items, int nsplit, float* grad);
}  // namespace sdfc

using namespace sdfc;

struct sdf_net {
  sdf_net_desc desc;
  int device = 0;
  int W = 0, L = 0, skip = 0, prec = 0;
  float bo = 0.0f;
  unsigned char* d_stream = nullptr;
  size_t stream_bytes = 0;
  int chunks_per_layer = 0;
  float* d_small = nullptr;
  float* d_scratch = nullptr;  // FP32 sigma stack, one slot per resident workgroup
  // FP32 handles: every call uses the one sigma stack, so calls on different
  // streams are ordered on the device: a call waits for the previous one when
  // that one ran on another stream (see fp32_order).
  hipEvent_t last_ev = nullptr;
  mutable hipStream_t last_stream = nullptr;
  mutable bool has_last = false;
  mutable std::mutex mu;
  int slots = 0;
  int variant = 0;            // tile variant of the 16-bit collide_project kernel (autotuner)
  float c_l1g = 0.0f, c_skg = 0.0f, c_wob = 0.0f;  // see KArgs
  float fsc[kLMax + 1] = {};  // FP8: forward / reverse operand-scale undo per layer
  float rsc[kLMax + 1] = {};
};

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(SDF_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// Checks the shape; fills W, L, skip.  Returns SDF_OK or an error code.
int check_desc(const sdf_net_desc* d, int* W, int* L, int* skip) {
  if (!d) return fail(SDF_EINVAL, "desc is NULL");
  if (d->n_hidden < 1 || d->n_hidden > SDF_MAX_HIDDEN)
    return fail(SDF_EINVAL, "n_hidden must be in [1, 16]");
  for (int i = 0; i < d->n_hidden; ++i)
    if (d->width[i] < 1) return fail(SDF_EINVAL, "widths must be positive");
  if (d->skip_layer == 1 || d->skip_layer < 0 || d->skip_layer > d->n_hidden)
    return fail(SDF_EINVAL, "skip_layer must be 0 or in [2, n_hidden]");
  if (!std::isfinite(d->beta) || d->beta <= 0.0f) return fail(SDF_EINVAL, "beta must be finite and > 0");
  if (d->fourier < 0 || d->fourier > 4096) return fail(SDF_EINVAL, "fourier must be in [0, 4096]");
  if (d->fourier > 0 && d->skip_layer != 0) return fail(SDF_EINVAL, "a Fourier-feature net has no skip input");
  if (d->precision != SDF_FP32 && d->precision != SDF_BF16 && d->precision != SDF_FP16 &&
      d->precision != SDF_BF16X3 && d->precision != SDF_FP8)
    return fail(SDF_EINVAL, "unknown precision");
  *W = d->width[0];
  *L = d->n_hidden;
  *skip = d->skip_layer;
  return SDF_OK;
}

int check_supported(int W, const sdf_net_desc* d) {
  for (int i = 1; i < d->n_hidden; ++i)
    if (d->width[i] != W) return fail(SDF_EUNSUPPORTED, "hidden widths must be equal");
  if (W != 64 && W != 128 && W != 256 && W != 512)
    return fail(SDF_EUNSUPPORTED, "width must be 64, 128, 256 or 512");
  if (W == 512 && d->precision == SDF_FP32)
    return fail(SDF_EUNSUPPORTED, "width 512 has 16-bit and FP8 kernels only");
  if (W < 128 && d->precision == SDF_FP8)
    return fail(SDF_EUNSUPPORTED, "FP8 needs width 128, 256 or 512 (K-blocks of 128)");
  if (d->fourier > 0 && (2 * d->fourier != W || d->precision == SDF_FP32 || d->precision == SDF_FP8))
    return fail(SDF_EUNSUPPORTED, "Fourier features need 2m == width and BF16, FP16 or BF16X3 operands");
  if (d->n_hidden < 2 || d->n_hidden > kLMax) return fail(SDF_EUNSUPPORTED, "depth must be in [2, 8]");
  return SDF_OK;
}

int64_t count_params(const sdf_net_desc* d) {
  int64_t c = 3 * (int64_t)d->fourier;  // B of the Fourier mapping
  int prev = d->fourier ? 2 * d->fourier : 3;
  for (int l = 1; l <= d->n_hidden; ++l) {
    const int w = d->width[l - 1];
    const int k = prev + (l == d->skip_layer ? 3 : 0);
    c += (int64_t)w * k + w;
    prev = w;
  }
  return c + prev + 1;
}

// Host view of the flat parameters.
struct Net {
  int W, L, skip, m;  // m: Fourier frequencies (0: the input is x itself)
  std::vector<const float*> Wl, bl;  // index l = 1..L
  const float* wo;
  float bo;
  const float* B;  // [m][3]
  int K(int l) const { return (l == 1 ? (m ? 2 * m : 3) : W) + (l == skip ? 3 : 0); }
};

Net view(const float* P, int W, int L, int skip, int m) {
  Net n{W, L, skip, m, std::vector<const float*>(L + 1), std::vector<const float*>(L + 1), nullptr, 0.0f, P};
  const float* q = P + 3 * (size_t)m;
  for (int l = 1; l <= L; ++l) {
    n.Wl[l] = q;
    q += (size_t)W * n.K(l);
    n.bl[l] = q;
    q += W;
  }
  n.wo = q;
  n.bo = q[W];
  return n;
}

uint16_t to_bf16(float v) {  // round to nearest even
  uint32_t u;
  std::memcpy(&u, &v, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffff) ? 0x40 : 0));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

uint16_t to_fp16(float v) {  // round to nearest even, saturating to +-inf on overflow
  return __builtin_bit_cast(uint16_t, (_Float16)v);
}

// float -> OCP E4M3 (bias 7, no infinities, largest finite 448), round to
// nearest even, saturated at +-448; values below 2^-10 in magnitude -> 0.
uint8_t to_e4m3(float v) {
  const uint8_t sign = std::signbit(v) ? 0x80 : 0x00;
  const double a = std::fabs((double)v);
  if (!(a == a)) return 0x7f;  // NaN
  if (a >= 448.0) return sign | 0x7e;
  int e;
  std::frexp(a, &e);  // a = m 2^e, m in [0.5, 1)
  int ex = e - 1;     // a in [2^ex, 2^(ex+1))
  if (ex < -6) ex = -6;  // subnormal range shares the 2^-6 exponent with a zero field
  const double q = std::nearbyint(std::ldexp(a, 3 - ex));  // units of 2^(ex-3), ties to even
  int mant = (int)q;
  int field = ex + 7;
  if (a < std::ldexp(1.0, -6)) {  // subnormal: value = mant 2^-9
    if (mant >= 8) return sign | 0x08;  // rounded up to 2^-6
    return sign | (uint8_t)mant;
  }
  if (mant >= 16) {  // rounded up to the next binade
    mant = 8;
    field += 1;
  }
  if (field > 15 || (field == 15 && mant - 8 > 6)) return sign | 0x7e;
  return sign | (uint8_t)((field << 3) | (mant - 8));
}

// Power-of-two exponent s with max |v| 2^s in (224, 448] (0 for an all-zero set).
int fp8_exponent(double maxabs) {
  if (!(maxabs > 0.0)) return 0;
  int s = (int)std::floor(std::log2(448.0 / maxabs));
  while (std::ldexp(maxabs, s) > 448.0) --s;
  if (s > 60) s = 60;
  if (s < -60) s = -60;
  return s;
}

// Per-layer power-of-two scales of the reverse-sweep vectors d_l (16-bit
// paths): S_l ~ -log2(rms(d_l)), estimated from the weights alone with
// rms(d_L) ~ rms(w_o)/2 and rms(d_{l-1}) ~ rms(d_l) |W_l|_F / sqrt(K) / 2.
std::vector<int> reverse_scales(const Net& n) {
  std::vector<int> S(n.L + 1, 0);
  double ss = 0.0;
  for (int j = 0; j < n.W; ++j) ss += (double)n.wo[j] * n.wo[j];
  double rms = 0.5 * std::sqrt(ss / n.W) + 1e-30;
  for (int l = n.L; l >= 1; --l) {
    S[l] = (int)std::lround(-std::log2(rms));
    if (S[l] > 100) S[l] = 100;
    if (S[l] < -100) S[l] = -100;
    if (l > 1) {
      double fro = 0.0;
      const int K = n.K(l);
      for (int j = 0; j < n.W; ++j)
        for (int k = 0; k < n.W; ++k) fro += (double)n.Wl[l][(size_t)j * K + k] * n.Wl[l][(size_t)j * K + k];
      rms = 0.5 * rms * std::sqrt(fro / n.W) + 1e-30;
    }
  }
  return S;
}

}  // namespace

extern "C" {

int64_t sdf_param_count(const sdf_net_desc* desc) {
  int W, L, skip;
  if (check_desc(desc, &W, &L, &skip) != SDF_OK) return -1;
  return count_params(desc);
}

const char* sdf_last_error(void) { return g_err.c_str(); }

int sdf_net_create(const sdf_net_desc* desc, const float* params, size_t n_params, int device,
                   sdf_net** out) {
  g_err.clear();
  if (!out) return fail(SDF_EINVAL, "out is NULL");
  *out = nullptr;
  int W, L, skip;
  int rc = check_desc(desc, &W, &L, &skip);
  if (rc) return rc;
  if (!params) return fail(SDF_EINVAL, "params is NULL");
  if ((int64_t)n_params != count_params(desc))
    return fail(SDF_EINVAL, "n_params is " + std::to_string(n_params) + ", expected " +
                                std::to_string(count_params(desc)));
  for (size_t i = 0; i < n_params; ++i)
    if (!std::isfinite(params[i])) return fail(SDF_EINVAL, "params must be finite");
  rc = check_supported(W, desc);
  if (rc) return rc;
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
  if (device < 0 || device >= ndev) return fail(SDF_EINVAL, "no such device");

  const int m = desc->fourier;
  const Net n = view(params, W, L, skip, m);
  const int prec = desc->precision;
  const double kappa = (double)desc->beta / std::log(2.0);  // beta * log2(e)
  std::vector<int> S = (prec == SDF_FP32) ? std::vector<int>(L + 1, 0) : reverse_scales(n);
  // FP8: weight exponents of the forward (sf) and reverse (sr) contraction of
  // every layer; forward activations enter the exchange as r / 4.
  std::vector<int> sf(L + 1, 0), sr(L + 1, 0);
  if (prec == SDF_FP8) {
    for (int l = 2; l <= L; ++l) {
      const int K = n.K(l);
      double mf = 0.0;
      for (int j = 0; j < W; ++j)
        for (int k = 0; k < W; ++k) mf = std::max(mf, std::fabs((double)n.Wl[l][(size_t)j * K + k]));
      sf[l] = fp8_exponent(mf);
      sr[l] = fp8_exponent(mf * std::ldexp(1.0, S[l - 1] - S[l]));
    }
  }
  // factor folded into the FP32 terms that are added to a scaled forward accumulator
  auto facc = [&](int l) { return prec == SDF_FP8 ? std::ldexp(1.0, sf[l] - 2) : 1.0; };

  // ---- small FP32 block ----
  const SmallLayout SL{W};
  std::vector<float> sm(SL.floats(), 0.0f);
  for (int j = 0; j < W; ++j) {
    if (m) {  // Fourier input: feature j = sin(2 pi (b . x + phase)), phase 1/4 for the cosines
      const float* b = n.B + 3 * (size_t)(j % m);
      for (int c = 0; c < 3; ++c) sm[SL.l1() + 4 * j + c] = b[c];
      sm[SL.l1() + 4 * j + 3] = j < m ? 0.0f : 0.25f;
      sm[SL.l1g() + j] = (float)(kappa * n.bl[1][j]);  // layer-1 bias of the MFMA layer
    } else {
      const float* w1 = n.Wl[1] + (size_t)j * n.K(1);
      for (int c = 0; c < 3; ++c) {
        sm[SL.l1() + 4 * j + c] = (float)(kappa * w1[c]);
        sm[SL.l1g() + 4 * j + c] = (float)std::ldexp((double)w1[c], -S[1]);
      }
      sm[SL.l1() + 4 * j + 3] = (float)(kappa * n.bl[1][j]);
    }
    if (skip) {
      const float* ws = n.Wl[skip] + (size_t)j * n.K(skip) + W;
      for (int c = 0; c < 3; ++c) {
        sm[SL.skf() + 4 * j + c] = (float)(kappa * ws[c] * facc(skip));
        sm[SL.skg() + 4 * j + c] = (float)std::ldexp((double)ws[c], -S[skip]);
      }
    }
    sm[SL.wof() + j] = (float)(n.wo[j] / kappa);
    sm[SL.wob() + j] = (float)std::ldexp((double)n.wo[j], S[L]);
    for (int l = 2; l <= L; ++l) sm[SL.bias(l) + j] = (float)(kappa * n.bl[l][j] * facc(l));
  }

  // ---- fragment stream: forward W_2..W_L, then reverse W_L^T..W_2^T ----
  std::vector<unsigned char> stream;
  int cpl = 0;
  auto emit16 = [&](auto at /* (row, col) -> float */) {
    // [wave][K-block][local M-tile][part] fragments: each wave reads one
    // contiguous slice holding the rows it owns (features [w W/4, (w+1) W/4)).
    // BF16x3 stores every weight as a pair hi = bf16(v), lo = bf16(v - hi).
    const int NWV = k16_waves(W);
    const int KB = W / 32, MTW = W / (16 * NWV), NS = (prec == SDF_BF16X3) ? 2 : 1;
    for (int w = 0; w < NWV; ++w)
      for (int kb = 0; kb < KB; ++kb)
        for (int ml = 0; ml < MTW; ++ml)
          for (int part = 0; part < NS; ++part)
            for (int lane = 0; lane < 64; ++lane) {
              const int g = lane >> 4, row = lane & 15, mt = MTW * w + ml;
              for (int e = 0; e < 8; ++e) {
                const int col = 32 * kb + 16 * (e / 4) + 4 * g + (e % 4);
                const float v = at(16 * mt + row, col);
                uint16_t h;
                if (prec == SDF_FP16) {
                  h = to_fp16(v);
                } else {
                  h = to_bf16(v);
                  if (part == 1) {
                    const uint32_t hb = (uint32_t)h << 16;
                    float hf;
                    std::memcpy(&hf, &hb, 4);
                    h = to_bf16(v - hf);
                  }
                }
                stream.push_back((unsigned char)(h & 0xff));
                stream.push_back((unsigned char)(h >> 8));
              }
            }
  };
  auto emit8 = [&](auto at, int sexp) {
    // [wave][K-block of 128][local M-tile] fragments of 64 lanes x 32 bytes:
    // lane 16 g + row, byte e holds A[16 mt + row][128 kb + 16 (e / 4) + 4 g + (e % 4)],
    // the features lane group g holds of M-tiles 8 kb .. 8 kb + 7.
    const int NWV = k16_waves(W);
    const int KB = W / 128, MTW = W / (16 * NWV);
    for (int w = 0; w < NWV; ++w)
      for (int kb = 0; kb < KB; ++kb)
        for (int ml = 0; ml < MTW; ++ml)
          for (int lane = 0; lane < 64; ++lane) {
            const int g = lane >> 4, row = lane & 15, mt = MTW * w + ml;
            for (int e = 0; e < 32; ++e) {
              const int col = 128 * kb + 16 * (e / 4) + 4 * g + (e % 4);
              stream.push_back(to_e4m3((float)std::ldexp((double)at(16 * mt + row, col), sexp)));
            }
          }
  };
  auto emit32 = [&](auto at) {
    const int MT = W / 16;
    for (int mt = 0; mt < MT; ++mt)
      for (int m = 0; m < MT; ++m)
        for (int lane = 0; lane < 64; ++lane) {
          const int g = lane >> 4, row = lane & 15;
          for (int i = 0; i < 4; ++i) {
            const float v = at(16 * mt + row, 16 * m + 4 * g + i);
            unsigned char b[4];
            std::memcpy(b, &v, 4);
            stream.insert(stream.end(), b, b + 4);
          }
        }
  };
  // Contractions on MFMA: layers 2..L, and layer 1 too for Fourier input
  // (K = 2m = W; its forward weights carry kappa since gamma is not rescaled).
  const int nf = m ? 1 : 2;
  for (int pass = 0; pass < 2; ++pass) {
    for (int step = 0; step < L - nf + 1; ++step) {
      const int l = pass == 0 ? nf + step : L - step;
      const float* Wl = n.Wl[l];
      const int K = n.K(l);
      const float sc = (float)std::ldexp(1.0, S[l - 1] - S[l]);
      const float fk = (l == 1) ? (float)kappa : 1.0f;
      auto fwd = [&](int r, int c) { return Wl[(size_t)r * K + c] * fk; };
      auto rev = [&](int r, int c) { return Wl[(size_t)c * K + r] * sc; };
      if (prec == SDF_FP32) {
        if (pass == 0) emit32(fwd); else emit32(rev);
      } else if (prec == SDF_FP8) {
        if (pass == 0) emit8(fwd, sf[l]); else emit8(rev, sr[l]);
      } else {
        if (pass == 0) emit16(fwd); else emit16(rev);
      }
    }
  }
  if (prec != SDF_FP32 && prec != SDF_FP8) {
    // a 16-bit value that overflowed would make every gradient through it infinite
    for (size_t i = 0; i + 1 < stream.size(); i += 2) {
      const uint16_t h = (uint16_t)(stream[i] | (stream[i + 1] << 8));
      const bool inf = (prec == SDF_FP16) ? ((h & 0x7c00) == 0x7c00) : ((h & 0x7f80) == 0x7f80);
      if (inf) return fail(SDF_EUNSUPPORTED, "a weight does not fit the 16-bit operand range");
    }
  }
  const size_t layer_bytes = (size_t)(W / 16) * (prec == SDF_FP32 ? W / 16 : W / 32) * kFrag;
  const size_t chunk = layer_bytes < 32768 ? layer_bytes : 32768;
  cpl = (int)(layer_bytes / chunk);

  int prev_dev = 0;
  (void)hipGetDevice(&prev_dev);
  if ((e = hipSetDevice(device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
  sdf_net* net = new sdf_net();
  net->desc = *desc;
  net->device = device;
  net->W = W;
  net->L = L;
  net->skip = skip;
  net->prec = prec;
  net->bo = n.bo;
  net->stream_bytes = stream.size();
  net->c_l1g = (float)(std::ldexp(1.0, -S[1]) / kappa);
  net->c_skg = skip ? (float)(std::ldexp(1.0, -S[skip]) / (kappa * facc(skip))) : 0.0f;
  net->c_wob = (float)(kappa * std::ldexp(1.0, S[L]));
  for (int l = 0; l <= kLMax; ++l) {
    net->fsc[l] = (prec == SDF_FP8 && l >= 2 && l <= L) ? (float)std::ldexp(1.0, 2 - sf[l]) : 1.0f;
    net->rsc[l] = (prec == SDF_FP8 && l >= 2 && l <= L) ? (float)std::ldexp(1.0, -sr[l]) : 1.0f;
  }
  net->chunks_per_layer = cpl;
  auto cleanup = [&](int code, const std::string& msg) {
    sdf_net_destroy(net);
    (void)hipSetDevice(prev_dev);
    return fail(code, msg);
  };
  // SDFC_FAIL_ALLOC=k (testing the out-of-memory path): the k-th device
  // allocation of this call reports failure without allocating.
  const char* fail_env = std::getenv("SDFC_FAIL_ALLOC");
  const int fail_at = fail_env ? std::atoi(fail_env) : 0;
  int n_alloc = 0;
  auto dev_alloc = [&](auto** p, size_t bytes) {
    if (++n_alloc == fail_at) return false;
    return hipMalloc((void**)p, bytes) == hipSuccess;
  };
  if (!dev_alloc(&net->d_stream, stream.size())) return cleanup(SDF_ENOMEM, "hipMalloc(stream)");
  if (!dev_alloc(&net->d_small, sm.size() * 4)) return cleanup(SDF_ENOMEM, "hipMalloc(small)");
  if (hipMemcpy(net->d_stream, stream.data(), stream.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(net->d_small, sm.data(), sm.size() * 4, hipMemcpyHostToDevice) != hipSuccess)
    return cleanup(SDF_EDEVICE, "hipMemcpy of packed weights");
  if (prec == SDF_FP32) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus < 1)
      return cleanup(SDF_EDEVICE, "hipDeviceGetAttribute(CU count)");
    net->slots = cus;  // one 4-wave workgroup per CU (LDS-bound)
    const size_t bytes = (size_t)net->slots * (kLMax - 1) * 4 * (W / 16) * 64 * 16;
    if (!dev_alloc(&net->d_scratch, bytes)) return cleanup(SDF_ENOMEM, "hipMalloc(scratch)");
    if (hipEventCreateWithFlags(&net->last_ev, hipEventDisableTiming) != hipSuccess)
      return cleanup(SDF_EDEVICE, "hipEventCreateWithFlags");
  }
  (void)hipSetDevice(prev_dev);
  *out = net;
  return SDF_OK;
}

int sdf_net_destroy(sdf_net* net) {
  if (!net) return SDF_OK;
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(net->device);
  if (net->d_stream) (void)hipFree(net->d_stream);
  if (net->d_small) (void)hipFree(net->d_small);
  if (net->d_scratch) (void)hipFree(net->d_scratch);
  if (net->last_ev) (void)hipEventDestroy(net->last_ev);
  (void)hipSetDevice(prev);
  delete net;
  return SDF_OK;
}

}  // extern "C"

namespace {

template <int MODE>
hipError_t launch(const sdf_net* net, const KArgs& a, hipStream_t s) {
  const int W = net->W;
  dim3 block(kBlock);
  if (net->prec == SDF_FP32) {
    dim3 grid((unsigned)(a.ntiles < net->slots ? a.ntiles : net->slots));
#define K32(WW) \
  if (W == WW) hipLaunchKernelGGL((sdf_k32<WW, MODE>), grid, block, 0, s, a);
    K32(64) K32(128) K32(256)
#undef K32
  } else {
    const bool pair = net->prec == SDF_BF16X3;  // points per workgroup, as in the kernel
    const int var = (MODE == MODE_PROJECT && k16_has_variant(W, net->prec == SDF_BF16 || net->prec == SDF_FP16))
                        ? net->variant : 0;
    const int64_t pts = k16_points(W, pair ? 2 : 1, net->prec == SDF_FP8, var);
    dim3 block16(64 * k16_waves(W));
    // a dispatch holds fewer than 2^32 work-items: split very large batches
    const int64_t max_pts = ((int64_t)1 << 22) * pts;
    for (int64_t p0 = 0; p0 < a.n; p0 += max_pts) {
      KArgs c = a;
      c.n = std::min<int64_t>(max_pts, a.n - p0);
      c.pts_in = a.pts_in + 3 * p0;
      c.pts_out = a.pts_out + 3 * p0;
      if (a.sdf) c.sdf = a.sdf + p0;
      if (a.grad) c.grad = a.grad + 3 * p0;
      if (a.normal) c.normal = a.normal + 3 * p0;
      if (a.hit) c.hit = a.hit + p0;
      dim3 grid((unsigned)((c.n + pts - 1) / pts));
#define K16(WW, PP) \
  if (W == WW && net->prec == PP && var == 0) hipLaunchKernelGGL((sdf_k16<WW, PP, MODE, 0>), grid, block16, 0, s, c);
      K16(64, PREC_BF16) K16(128, PREC_BF16) K16(256, PREC_BF16)
      K16(64, PREC_FP16) K16(128, PREC_FP16) K16(256, PREC_FP16)
      K16(64, PREC_BF16X3) K16(128, PREC_BF16X3) K16(256, PREC_BF16X3)
      K16(512, PREC_BF16) K16(512, PREC_FP16) K16(512, PREC_BF16X3)
      K16(128, PREC_FP8) K16(256, PREC_FP8) K16(512, PREC_FP8)
#undef K16
      if constexpr (MODE == MODE_PROJECT) {
#define K16V(WW, PP) \
  if (W == WW && net->prec == PP && var == 1) hipLaunchKernelGGL((sdf_k16<WW, PP, MODE, 1>), grid, block16, 0, s, c);
        K16V(128, PREC_BF16) K16V(256, PREC_BF16) K16V(512, PREC_BF16)
        K16V(128, PREC_FP16) K16V(256, PREC_FP16) K16V(512, PREC_FP16)
#undef K16V
      }
    }
  }
  return hipGetLastError();
}

bool aligned4(const void* p) { return ((uintptr_t)p & 3u) == 0; }

// Shared checks and launch for the three query entry points.
template <int MODE>
int run(const sdf_net* net, const float* pts_in, float* pts_out, int64_t n, float eps, float* sdf,
        float* grad, float* normal, uint8_t* hit, void* stream, const float* T = nullptr) {
  g_err.clear();
  if (!net) return fail(SDF_EINVAL, "net is NULL");
  KArgs a{};
  if (T) {  // collider frame T = [A t; 0 1] (host, row-major)
    for (int i = 0; i < 16; ++i)
      if (!std::isfinite(T[i])) return fail(SDF_EINVAL, "T must be finite");
    if (std::fabs(T[12]) > 1e-6f || std::fabs(T[13]) > 1e-6f || std::fabs(T[14]) > 1e-6f ||
        std::fabs(T[15] - 1.0f) > 1e-6f)
      return fail(SDF_EINVAL, "the last row of T must be (0, 0, 0, 1)");
    const double m[3][3] = {{T[0], T[1], T[2]}, {T[4], T[5], T[6]}, {T[8], T[9], T[10]}};
    const double det = m[0][0] * (m[1][1] * m[2][2] - m[1][2] * m[2][1]) -
                       m[0][1] * (m[1][0] * m[2][2] - m[1][2] * m[2][0]) +
                       m[0][2] * (m[1][0] * m[2][1] - m[1][1] * m[2][0]);
    double scale = 0.0;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) scale = std::max(scale, std::fabs(m[i][j]));
    if (!(std::fabs(det) > 1e-9 * scale * scale * scale)) return fail(SDF_EINVAL, "T is singular");
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {  // adjugate / det
        const int r0 = (j + 1) % 3, r1 = (j + 2) % 3, c0 = (i + 1) % 3, c1 = (i + 2) % 3;
        a.Ai[3 * i + j] = (float)((m[r0][c0] * m[r1][c1] - m[r0][c1] * m[r1][c0]) / det);
      }
    a.tr[0] = T[3];
    a.tr[1] = T[7];
    a.tr[2] = T[11];
    a.rigid = 1;
  }
  if (n < 0) return fail(SDF_EINVAL, "n < 0");
  if (MODE == MODE_PROJECT && !std::isfinite(eps)) return fail(SDF_EINVAL, "eps must be finite");
  if (n == 0) return SDF_OK;  // pointers may be NULL for an empty batch
  if (!pts_in) return fail(SDF_EINVAL, "pts is NULL");
  if (MODE == MODE_QUERY && !sdf) return fail(SDF_EINVAL, "sdf is NULL");
  if (MODE == MODE_GRAD && !grad) return fail(SDF_EINVAL, "grad is NULL");
  if (!aligned4(pts_in) || !aligned4(sdf) || !aligned4(grad) || !aligned4(normal))
    return fail(SDF_EINVAL, "float arrays must be 4-byte aligned");
  if (n > ((int64_t)1 << 40)) return fail(SDF_EINVAL, "n too large");
  if (n == 0) return SDF_OK;
  const int64_t tiles = (n + kPtsPerBlock - 1) / kPtsPerBlock;
  if (2 * tiles > 0x7fffffff) return fail(SDF_EINVAL, "n too large");
  a.pts_in = pts_in;
  a.pts_out = pts_out;
  a.n = n;
  a.sdf = sdf;
  a.grad = grad;
  a.normal = normal;
  a.hit = hit;
  a.eps = eps;
  a.bo = net->bo;
  a.stream = net->d_stream;
  a.small = net->d_small;
  a.scratch = net->d_scratch;
  for (int l = 0; l <= kLMax; ++l) {
    a.fsc[l] = net->fsc[l];
    a.rsc[l] = net->rsc[l];
  }
  a.L = net->L;
  a.skip = net->skip;
  a.ff = net->desc.fourier > 0 ? 1 : 0;
  a.c_l1g = net->c_l1g;
  a.c_skg = net->c_skg;
  a.c_wob = net->c_wob;
  a.nch = (net->L - 1) * net->chunks_per_layer * (MODE == MODE_QUERY ? 1 : 2);
  a.ntiles = (int)tiles;
  int prev = 0;
  (void)hipGetDevice(&prev);
  if (prev != net->device) (void)hipSetDevice(net->device);
  hipError_t e = hipSuccess;
  if (net->prec == SDF_FP32) {
    // One sigma stack per handle: order this call after the previous one if
    // that ran on another stream.  A stream under capture is left alone (the
    // header asks captured FP32 calls on one handle to use one stream).
    const hipStream_t s = (hipStream_t)stream;
    std::lock_guard<std::mutex> lock(net->mu);
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    e = hipStreamIsCapturing(s, &cs);
    const bool eager = e == hipSuccess && cs == hipStreamCaptureStatusNone;
    if (e == hipSuccess && eager && net->has_last && net->last_stream != s)
      e = hipStreamWaitEvent(s, net->last_ev, 0);
    if (e == hipSuccess) e = launch<MODE>(net, a, s);
    if (e == hipSuccess && eager) {
      e = hipEventRecord(net->last_ev, s);
      net->last_stream = s;
      net->has_last = true;
    }
  } else {
    e = launch<MODE>(net, a, (hipStream_t)stream);
  }
  if (prev != net->device) (void)hipSetDevice(prev);
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  return SDF_OK;
}

}  // namespace

extern "C" {

int sdf_query(const sdf_net* net, const float* pts, int64_t n, float* sdf, void* stream) {
  return run<MODE_QUERY>(net, pts, nullptr, n, 0.0f, sdf, nullptr, nullptr, nullptr, stream);
}

int sdf_query_grad(const sdf_net* net, const float* pts, int64_t n, float* sdf, float* grad,
                   void* stream) {
  return run<MODE_GRAD>(net, pts, nullptr, n, 0.0f, sdf, grad, nullptr, nullptr, stream);
}

int collide_project(const sdf_net* net, float* pts, int64_t n, float eps, float* sdf,
                    float* normal, uint8_t* hit, void* stream) {
  return run<MODE_PROJECT>(net, pts, pts, n, eps, sdf, nullptr, normal, hit, stream);
}

int sdf_query_rigid(const sdf_net* net, const float* T, const float* pts, int64_t n, float* sdf,
                    void* stream) {
  if (!T) return fail(SDF_EINVAL, "T is NULL");
  return run<MODE_QUERY>(net, pts, nullptr, n, 0.0f, sdf, nullptr, nullptr, nullptr, stream, T);
}

int sdf_query_grad_rigid(const sdf_net* net, const float* T, const float* pts, int64_t n, float* sdf,
                         float* grad, void* stream) {
  if (!T) return fail(SDF_EINVAL, "T is NULL");
  return run<MODE_GRAD>(net, pts, nullptr, n, 0.0f, sdf, grad, nullptr, nullptr, stream, T);
}

int collide_project_rigid(const sdf_net* net, const float* T, float* pts, int64_t n, float eps,
                          float* sdf, float* normal, uint8_t* hit, void* stream) {
  if (!T) return fail(SDF_EINVAL, "T is NULL");
  return run<MODE_PROJECT>(net, pts, pts, n, eps, sdf, nullptr, normal, hit, stream, T);
}

}  // extern "C"

// ------------------------------------------------------------------ fitting

namespace {

constexpr int64_t kTrainChunk = 65536;  // points per chunk of a fitting step

struct TrainLayout {  // byte offsets inside the caller's workspace
  size_t stream, small, scratch, E, H, U, loss, part, total;
  int64_t chunk;
  int items, nsplit;  // weight-gradient work items and point slices per item
};

// Output blocks of the weight-gradient contraction (wgrad_kernel): 128 x 128
// from width 128 (eight waves), 64 x 64 below.
int wgrad_bs(int W) { return W >= 128 ? 128 : 64; }

// Work items of the weight-gradient contraction: row blocks of every layer
// times column blocks plus the 16-wide tail block.
int wgrad_items(int W, int L) {
  const int RB = W / wgrad_bs(W), CB = RB + 1;
  return RB + (L - 1) * RB * CB + CB;
}

}  // namespace

constexpr size_t kStaticScratchBytes = (size_t)64 << 20;  // 64 MiB per device
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

// Chunk of a batch of n points for a workspace sized for at most max_chunk.
int64_t train_chunk(int64_t n, int64_t max_chunk) { return n < max_chunk ? (n > 0 ? n : 1) : max_chunk; }

// nsplit: point slices of the weight-gradient contraction (1: no partial
// buffer, the slices' sums go straight into the gradient).
TrainLayout train_layout(int W, int L, int64_t chunk, int slots, int nsplit) {
  TrainLayout t{};
  auto up = [](size_t v) { return (v + 255) & ~(size_t)255; };
  t.items = wgrad_items(W, L);
  t.nsplit = nsplit;
  size_t o = 0;
  t.stream = o;
  o = up(o + 2 * (size_t)(L - 1) * (W / 16) * (W / 16) * kFrag);
  t.small = o;
  o = up(o + (size_t)SmallLayout{W}.floats() * 4);
  t.scratch = o;
  o = up(o + (size_t)slots * (kLMax - 1) * 4 * (W / 16) * 64 * 16);
  t.E = o;
  o = up(o + (size_t)L * chunk * W * 4);
  t.H = o;
  o = up(o + (size_t)(L + 1) * chunk * (W + 16) * 4);
  t.U = o;
  o = up(o + (size_t)chunk * 16 * 4);
  t.loss = o;
  o = up(o + (size_t)chunk * 4);
  t.part = o;
  if (nsplit > 1) o = up(o + (size_t)nsplit * t.items * wgrad_bs(W) * wgrad_bs(W) * 4);
  t.total = o;
  t.chunk = chunk;
  return t;
}

// Point slices per weight-gradient work item: enough workgroups to fill the
// GPU a few times over, slices of at least 1024 points of a full chunk.
int wgrad_splits(int W, int L, int cus) {
  const int s = (wgrad_bs(W) == 128 ? 4 : 8) * cus / wgrad_items(W, L);
  return s < 1 ? 1 : (s > 64 ? 64 : s);
}

int train_check(const sdf_net_desc* desc, int* W, int* L, int* skip) {
  int rc = check_desc(desc, W, L, skip);
  if (rc) return rc;
  rc = check_supported(*W, desc);
  if (rc) return rc;
  if (desc->precision != SDF_FP32) return fail(SDF_EUNSUPPORTED, "fitting runs in FP32 (precision must be SDF_FP32)");
  if (desc->fourier) return fail(SDF_EUNSUPPORTED, "fitting takes networks without Fourier input");
  return SDF_OK;
}

int device_cus(int* cus) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  e = hipDeviceGetAttribute(cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess || *cus < 1) return fail(SDF_EDEVICE, "hipDeviceGetAttribute(CU count)");
  return SDF_OK;
}

int train_args(const sdf_net_desc* desc, const float* params, const float* pts, const float* target,
               int64_t n, float delta, const float* grad_params, const float* loss, int* W, int* L,
               int* skip) {
  int rc = train_check(desc, W, L, skip);
  if (rc) return rc;
  if (!params || !grad_params || !loss || (n > 0 && (!pts || !target)))
    return fail(SDF_EINVAL, "NULL pointer argument");
  if (n < 0) return fail(SDF_EINVAL, "n < 0");
  if (!std::isfinite(delta) || delta <= 0.0f) return fail(SDF_EINVAL, "delta must be finite and > 0");
  if (!aligned4(params) || !aligned4(pts) || !aligned4(target) || !aligned4(grad_params) || !aligned4(loss))
    return fail(SDF_EINVAL, "arrays must be 4-byte aligned");
  if (n > ((int64_t)1 << 40)) return fail(SDF_EINVAL, "n too large");
  return SDF_OK;
}

// One fitting step over n points, chunk by chunk, in the workspace `ws` laid
// out as `lay`; the persistent tile kernel runs at most `slots` workgroups
// (its sigma stack has that many slots).
int train_run(const sdf_net_desc* desc, int W, int L, int skip, const float* params, const float* pts,
              const float* target, int64_t n, float delta, float* grad_params, float* loss,
              unsigned char* ws, const TrainLayout& lay, int slots, hipStream_t s) {
  const int64_t np = count_params(desc);
  TrainNet t{};
  t.W = W;
  t.L = L;
  t.skip = skip;
  t.kappa = (float)((double)desc->beta / std::log(2.0));
  {
    int64_t o = 0;
    int prev = 3;
    for (int l = 1; l <= L; ++l) {
      const int k = prev + (l == skip ? 3 : 0);
      t.offW[l] = o;
      o += (int64_t)W * k;
      t.offb[l] = o;
      o += W;
      prev = W;
    }
    t.offo = o;
  }
  hipLaunchKernelGGL(fill_kernel, dim3(1024), dim3(256), 0, s, grad_params, np, 0.0f);
  hipLaunchKernelGGL(fill_kernel, dim3(1), dim3(64), 0, s, loss, (int64_t)1, 0.0f);
  if (n == 0) {
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? SDF_OK : hip_fail(e, "kernel launch");
  }
  float* d_stream = (float*)(ws + lay.stream);
  float* d_small = (float*)(ws + lay.small);
  hipLaunchKernelGGL(pack_fp32_kernel, dim3(2048), dim3(256), 0, s, t, params, d_stream, d_small);

  KArgs a{};
  a.stream = (const unsigned char*)d_stream;
  a.small = d_small;
  a.scratch = (float*)(ws + lay.scratch);
  a.L = L;
  a.skip = skip;
  a.nch = (L - 1) * (int)((size_t)(W / 16) * (W / 16) * kFrag / std::min<size_t>((size_t)(W / 16) * (W / 16) * kFrag, 32768)) * 2;
  a.ws_E = (float*)(ws + lay.E);
  a.ws_H = (float*)(ws + lay.H);
  a.ws_U = (float*)(ws + lay.U);
  a.ws_loss = (float*)(ws + lay.loss);
  a.bo_dev = params + t.offo + W;
  a.delta = delta;
  a.inv_n = (float)(1.0 / (double)n);
  a.inv_kappa = 1.0f / t.kappa;
  const int items = lay.items, nsplit = lay.nsplit;
  float* part = (float*)(ws + lay.part);
  for (int64_t c0 = 0; c0 < n; c0 += lay.chunk) {
    const int64_t cn = std::min<int64_t>(lay.chunk, n - c0);
    a.pts_in = pts + 3 * c0;
    a.target = target + c0;
    a.n = cn;
    a.ntiles = (int)((cn + kPtsPerBlock - 1) / kPtsPerBlock);
    dim3 grid((unsigned)std::min<int64_t>(a.ntiles, slots));
#define KT(WW) \
  if (W == WW) hipLaunchKernelGGL((sdf_k32<WW, MODE_TRAIN>), grid, dim3(kBlock), 0, s, a);
    KT(64) KT(128) KT(256)
#undef KT
    const int bs = wgrad_bs(W);
    if (bs == 128)
      hipLaunchKernelGGL(wgrad_kernel<128>, dim3(items * nsplit), dim3(128 * 128 / 32), 0, s, t, a.ws_E, a.ws_H,
                         a.ws_U, cn, items, nsplit, part, grad_params);
    else
      hipLaunchKernelGGL(wgrad_kernel<64>, dim3(items * nsplit), dim3(64 * 64 / 32), 0, s, t, a.ws_E, a.ws_H,
                         a.ws_U, cn, items, nsplit, part, grad_params);
    if (nsplit > 1) {
      const dim3 rg((unsigned)(((int64_t)items * bs * bs + 255) / 256));
      if (bs == 128)
        hipLaunchKernelGGL(wgrad_reduce_kernel<128>, rg, dim3(256), 0, s, t, part, items, nsplit, grad_params);
      else
        hipLaunchKernelGGL(wgrad_reduce_kernel<64>, rg, dim3(256), 0, s, t, part, items, nsplit, grad_params);
    }
    hipLaunchKernelGGL(loss_reduce_kernel, dim3(1), dim3(1024), 0, s, a.ws_loss, cn, loss);
  }
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? SDF_OK : hip_fail(e, "kernel launch");
}

// ---- the static scratch of sdf_train_step_noalloc (callers that cannot allocate)
//
// `scratch` (file scope, below) is a fixed array in the code object: every GPU
// the library runs on holds its own copy until the process ends.  Host code
// never uses the array's name as an address: its device address is looked up
// once per device with hipGetSymbolAddress (with that device current) and
// kept in g_scratch_ptr, which is what the kernels receive.
constexpr int kStaticSlots = 32;  // workgroups of the persistent tile kernel (sigma-stack slots)
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[kMaxDevices] = {};

int static_scratch(int dev, unsigned char** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(SDF_EUNSUPPORTED, "device index beyond the static scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[dev] = (unsigned char*)p;
  }
  *out = g_scratch_ptr[dev];
  return SDF_OK;
}

}  // namespace

extern "C" {

int64_t sdf_train_workspace_bytes(const sdf_net_desc* desc, int64_t n) {
  g_err.clear();
  int W, L, skip, cus;
  if (train_check(desc, &W, &L, &skip) != SDF_OK || n < 0) return -1;
  if (device_cus(&cus) != SDF_OK) return -1;
  return (int64_t)train_layout(W, L, train_chunk(n, kTrainChunk), cus, wgrad_splits(W, L, cus)).total;
}

int sdf_train_step(const sdf_net_desc* desc, const float* params, const float* pts,
                   const float* target, int64_t n, float delta, float* grad_params, float* loss,
                   void* workspace, size_t workspace_bytes, void* stream) {
  g_err.clear();
  int W, L, skip;
  int rc = train_args(desc, params, pts, target, n, delta, grad_params, loss, &W, &L, &skip);
  if (rc) return rc;
  if (n > 0 && !workspace) return fail(SDF_EINVAL, "NULL pointer argument");
  if ((uintptr_t)workspace & 255u) return fail(SDF_EINVAL, "the workspace must be 256-byte aligned");
  int cus;
  rc = device_cus(&cus);
  if (rc) return rc;
  const TrainLayout lay = train_layout(W, L, train_chunk(n, kTrainChunk), cus, wgrad_splits(W, L, cus));
  if (n > 0 && workspace_bytes < lay.total)
    return fail(SDF_EINVAL, "workspace too small: need " + std::to_string(lay.total) + " bytes");
  return train_run(desc, W, L, skip, params, pts, target, n, delta, grad_params, loss,
                   (unsigned char*)workspace, lay, cus, (hipStream_t)stream);
}

int sdf_train_step_noalloc(const sdf_net_desc* desc, const float* params, const float* pts,
                           const float* target, int64_t n, float delta, float* grad_params,
                           float* loss, void* stream) {
  g_err.clear();
  int W, L, skip;
  int rc = train_args(desc, params, pts, target, n, delta, grad_params, loss, &W, &L, &skip);
  if (rc) return rc;
  int dev = 0;
  const hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  unsigned char* ws = nullptr;
  rc = static_scratch(dev, &ws);
  if (rc) return rc;
  int cus;
  rc = device_cus(&cus);
  if (rc) return rc;
  const int slots = std::min(cus, kStaticSlots);
  // the largest chunk (a multiple of the tile) whose workspace fits the scratch
  int64_t chunk = std::min<int64_t>(train_chunk(n, kTrainChunk), kTrainChunk);
  chunk = (chunk + kPtsPerBlock - 1) / kPtsPerBlock * kPtsPerBlock;
  while (chunk > kPtsPerBlock && train_layout(W, L, chunk, slots, 1).total > kStaticScratchBytes)
    chunk -= kPtsPerBlock;
  const TrainLayout lay = train_layout(W, L, chunk, slots, 1);
  if (lay.total > kStaticScratchBytes)
    return fail(SDF_EUNSUPPORTED, "network too large for the static scratch: one tile needs " +
                                      std::to_string(lay.total) + " bytes of " +
                                      std::to_string(kStaticScratchBytes));
  return train_run(desc, W, L, skip, params, pts, target, n, delta, grad_params, loss, ws, lay, slots,
                   (hipStream_t)stream);
}

}  // extern "C"

// ------------------------------------------------------------ grouped calls

struct sdf_group {
  int device = 0;
  int prec = 0;
  int mode = SDF_GROUP_PER_WIDTH;  // SDF_GROUP_*: how a pass is launched
  // persistent launch (all members of width >= 128, at most 512 of them):
  // members in work order, their widths, their first work items (n + 1), the
  // two work counters; one workgroup per CU
  bool persist_ok = false;
  int cus = 0, n_persist = 0;
  KArgs* d_pargs = nullptr;
  int* d_pwidth = nullptr;
  int* d_pstart = nullptr;
  int* d_ctr = nullptr;
  struct Class {
    int W = 0, n = 0, var = 0;
    int tiles[2] = {0, 0};         // per tile variant
    KArgs* d_args = nullptr;       // [n]
    int* d_start[2] = {nullptr, nullptr};  // [n] per tile variant
  };
  std::vector<Class> classes;
  std::vector<const sdf_net*> nets;  // members with vertices, class by class
  std::vector<KArgs> args;           // host copy of the device table, same order
  void* d_mem = nullptr;
};

namespace {

bool has_variant(int W, int prec) { return k16_has_variant(W, prec == SDF_BF16 || prec == SDF_FP16); }

// One grouped launch for a width class with the given tables and tile variant.
hipError_t launch_class(int prec, const sdf_group::Class& c, const KArgs* d_args, const int* d_start,
                        int var, hipStream_t s) {
  const int tiles = c.tiles[var];
  const dim3 block(64 * k16_waves(c.W));
  // a dispatch holds fewer than 2^32 work-items
  for (int64_t t0 = 0; t0 < tiles; t0 += 1 << 22) {
    const dim3 grid((unsigned)std::min<int64_t>(1 << 22, tiles - t0));
#define KG(WW, PP, VV)                                                                               \
  if (c.W == WW && prec == PP && var == VV)                                                          \
    hipLaunchKernelGGL((sdf_k16_group<WW, PP, MODE_PROJECT, VV>), grid, block, 0, s, d_args, d_start, \
                       c.n, (int)t0);
    KG(64, PREC_BF16, 0) KG(128, PREC_BF16, 0) KG(256, PREC_BF16, 0) KG(512, PREC_BF16, 0)
    KG(64, PREC_FP16, 0) KG(128, PREC_FP16, 0) KG(256, PREC_FP16, 0) KG(512, PREC_FP16, 0)
    KG(64, PREC_BF16X3, 0) KG(128, PREC_BF16X3, 0) KG(256, PREC_BF16X3, 0) KG(512, PREC_BF16X3, 0)
    KG(128, PREC_FP8, 0) KG(256, PREC_FP8, 0) KG(512, PREC_FP8, 0)
    KG(128, PREC_BF16, 1) KG(256, PREC_BF16, 1) KG(512, PREC_BF16, 1)
    KG(128, PREC_FP16, 1) KG(256, PREC_FP16, 1) KG(512, PREC_FP16, 1)
#undef KG
  }
  return hipGetLastError();
}

// The persistent launch over tables (members in work order) with counters ctr.
hipError_t launch_persist(int prec, int cus, const KArgs* d_args, const int* d_width, const int* d_start, int n,
                          int* d_ctr, hipStream_t s) {
  const dim3 grid((unsigned)cus), block(512);
#define KP(PP) \
  if (prec == PP) hipLaunchKernelGGL((sdf_k16_persist<PP>), grid, block, 0, s, d_args, d_width, d_start, n, d_ctr);
  KP(PREC_BF16) KP(PREC_FP16) KP(PREC_BF16X3) KP(PREC_FP8)
#undef KP
  return hipGetLastError();
}

// A whole pass: one persistent launch, every class (grouped) or every network
// (per network), with the class tables at `d_args`-relative positions of the
// group (off) or host args.
hipError_t group_pass(const sdf_group* grp, const KArgs* d_table, const std::vector<KArgs>& host_args,
                      hipStream_t s) {
  if (grp->mode == SDF_GROUP_PERSISTENT)
    return launch_persist(grp->prec, grp->cus, grp->d_pargs, grp->d_pwidth, grp->d_pstart, grp->n_persist,
                          grp->d_ctr, s);
  if (grp->mode == SDF_GROUP_PER_NETWORK) {
    for (size_t i = 0; i < grp->nets.size(); ++i) {
      const hipError_t e = launch<MODE_PROJECT>(grp->nets[i], host_args[i], s);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  int off = 0;
  for (const auto& c : grp->classes) {
    const hipError_t e = launch_class(grp->prec, c, d_table + off, c.d_start[c.var], c.var, s);
    if (e != hipSuccess) return e;
    off += c.n;
  }
  return hipSuccess;
}

// Mean milliseconds of `reps` calls of fn after one warm-up call.
template <class F>
float time_ms(F fn, hipStream_t s, int reps) {
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return -1.0f;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return -1.0f;
  }
  fn();
  (void)hipEventRecord(e0, s);
  for (int r = 0; r < reps; ++r) fn();
  (void)hipEventRecord(e1, s);
  (void)hipEventSynchronize(e1);
  float ms = -1.0f;
  (void)hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return ms / reps;
}

}  // namespace

extern "C" {

int sdf_group_destroy(sdf_group* grp) {
  if (!grp) return SDF_OK;
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(grp->device);
  if (grp->d_mem) (void)hipFree(grp->d_mem);
  (void)hipSetDevice(prev);
  delete grp;
  return SDF_OK;
}

int sdf_group_create(const sdf_net* const* nets, int n_nets, float* const* pts, const int64_t* counts,
                     float eps, sdf_group** out) {
  g_err.clear();
  if (!out) return fail(SDF_EINVAL, "out is NULL");
  *out = nullptr;
  if (!nets || !pts || !counts || n_nets < 1 || n_nets > 4096)
    return fail(SDF_EINVAL, "need 1..4096 networks with vertex buffers and counts");
  if (!std::isfinite(eps)) return fail(SDF_EINVAL, "eps must be finite");
  const int dev = nets[0] ? nets[0]->device : 0;
  const int prec = nets[0] ? nets[0]->prec : 0;
  for (int i = 0; i < n_nets; ++i) {
    if (!nets[i]) return fail(SDF_EINVAL, "a network handle is NULL");
    if (nets[i]->device != dev) return fail(SDF_EINVAL, "all networks must live on one device");
    if (nets[i]->prec != prec) return fail(SDF_EINVAL, "all networks must share one precision");
    if (counts[i] < 0 || counts[i] > ((int64_t)1 << 31)) return fail(SDF_EINVAL, "bad vertex count");
    if (counts[i] > 0 && (!pts[i] || !aligned4(pts[i]))) return fail(SDF_EINVAL, "bad vertex buffer");
  }
  if (prec == SDF_FP32) return fail(SDF_EUNSUPPORTED, "grouped launches run the 16-bit kernels only");
  const bool pair = prec == SDF_BF16X3;
  auto pts_per_tile = [&](int W, int var) { return k16_points(W, pair ? 2 : 1, prec == SDF_FP8, var); };

  sdf_group* grp = new sdf_group();
  grp->device = dev;
  grp->prec = prec;
  std::vector<int> starts[2];
  const int widths[4] = {64, 128, 256, 512};
  for (int W : widths) {
    std::vector<int> idx;
    for (int i = 0; i < n_nets; ++i)
      if (nets[i]->W == W && counts[i] > 0) idx.push_back(i);
    if (idx.empty()) continue;
    // longest tiles first (deeper networks, then larger patches)
    std::sort(idx.begin(), idx.end(), [&](int a, int b) {
      if (nets[a]->L != nets[b]->L) return nets[a]->L > nets[b]->L;
      return counts[a] > counts[b];
    });
    sdf_group::Class c;
    c.W = W;
    c.n = (int)idx.size();
    int64_t tiles[2] = {0, 0};
    for (int i : idx) {
      const sdf_net* net = nets[i];
      KArgs a{};
      a.pts_in = pts[i];
      a.pts_out = pts[i];
      a.n = counts[i];
      a.eps = eps;
      a.bo = net->bo;
      a.stream = net->d_stream;
      a.small = net->d_small;
      a.L = net->L;
      a.skip = net->skip;
      a.ff = net->desc.fourier > 0 ? 1 : 0;
      a.c_l1g = net->c_l1g;
      a.c_skg = net->c_skg;
      a.c_wob = net->c_wob;
      for (int l = 0; l <= kLMax; ++l) {
        a.fsc[l] = net->fsc[l];
        a.rsc[l] = net->rsc[l];
      }
      for (int v = 0; v < 2; ++v) {
        starts[v].push_back((int)tiles[v]);
        tiles[v] += (counts[i] + pts_per_tile(W, v) - 1) / pts_per_tile(W, v);
      }
      grp->args.push_back(a);
      grp->nets.push_back(net);
    }
    if (tiles[1] > 0x7fffffff) {
      sdf_group_destroy(grp);
      return fail(SDF_EINVAL, "too many tiles");
    }
    c.tiles[0] = (int)tiles[0];
    c.tiles[1] = (int)tiles[1];
    grp->classes.push_back(c);
  }
  // Persistent work order: members by decreasing cost of one tile (width^2 x
  // depth x points per tile), then larger patches first; tile variant 0.
  const int nm = (int)grp->args.size();
  std::vector<int> order(nm);
  for (int i = 0; i < nm; ++i) order[i] = i;
  auto tile_cost = [&](int i) {
    const sdf_net* n = grp->nets[i];
    return (double)n->W * n->W * n->L * pts_per_tile(n->W, 0);
  };
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
    if (tile_cost(x) != tile_cost(y)) return tile_cost(x) > tile_cost(y);
    return grp->args[x].n > grp->args[y].n;
  });
  std::vector<KArgs> pargs;
  std::vector<int> pwidth, pstart(1, 0);
  bool persist_ok = nm > 0 && nm <= 512;  // the kernel keeps the item table in LDS
  for (int q = 0; q < nm; ++q) {
    const int i = order[q];
    const int W = grp->nets[i]->W;
    const int64_t next = pstart.back() + (grp->args[i].n + pts_per_tile(W, 0) - 1) / pts_per_tile(W, 0);
    persist_ok = persist_ok && W >= 128 && next < 0x7fffffff;
    pargs.push_back(grp->args[i]);
    pwidth.push_back(W);
    pstart.push_back((int)std::min<int64_t>(next, 0x7fffffff));
  }
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(dev);
  if (hipDeviceGetAttribute(&grp->cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || grp->cus < 1) {
    (void)hipSetDevice(prev);
    sdf_group_destroy(grp);
    return fail(SDF_EDEVICE, "hipDeviceGetAttribute(CU count)");
  }
  auto up = [](size_t v) { return (v + 255) & ~(size_t)255; };
  const size_t abytes = grp->args.size() * sizeof(KArgs), sbytes = starts[0].size() * sizeof(int);
  const size_t o_pargs = up(abytes + 2 * sbytes), o_pwidth = up(o_pargs + abytes),
               o_pstart = up(o_pwidth + nm * sizeof(int)), o_ctr = up(o_pstart + (nm + 1) * sizeof(int)),
               total = o_ctr + 256;
  if (!grp->args.empty()) {
    if (hipMalloc(&grp->d_mem, total) != hipSuccess) {
      (void)hipSetDevice(prev);
      sdf_group_destroy(grp);
      return fail(SDF_ENOMEM, "hipMalloc(group tables)");
    }
    unsigned char* m = (unsigned char*)grp->d_mem;
    if (hipMemcpy(m, grp->args.data(), abytes, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(m + abytes, starts[0].data(), sbytes, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(m + abytes + sbytes, starts[1].data(), sbytes, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(m + o_pargs, pargs.data(), abytes, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(m + o_pwidth, pwidth.data(), nm * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(m + o_pstart, pstart.data(), (nm + 1) * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(m + o_ctr, 0, 256) != hipSuccess) {
      (void)hipSetDevice(prev);
      sdf_group_destroy(grp);
      return fail(SDF_EDEVICE, "hipMemcpy(group tables)");
    }
    int off = 0;
    for (auto& c : grp->classes) {
      c.d_args = (KArgs*)m + off;
      c.d_start[0] = (int*)(m + abytes) + off;
      c.d_start[1] = (int*)(m + abytes + sbytes) + off;
      off += c.n;
    }
    grp->d_pargs = (KArgs*)(m + o_pargs);
    grp->d_pwidth = (int*)(m + o_pwidth);
    grp->d_pstart = (int*)(m + o_pstart);
    grp->d_ctr = (int*)(m + o_ctr);
    grp->n_persist = nm;
    grp->persist_ok = persist_ok;
    grp->mode = SDF_GROUP_PER_WIDTH;
  }
  (void)hipSetDevice(prev);
  *out = grp;
  return SDF_OK;
}

int sdf_group_set_launch(sdf_group* grp, int mode) {
  g_err.clear();
  if (!grp) return fail(SDF_EINVAL, "group is NULL");
  if (mode != SDF_GROUP_PER_WIDTH && mode != SDF_GROUP_PER_NETWORK && mode != SDF_GROUP_PERSISTENT)
    return fail(SDF_EINVAL, "unknown launch mode");
  if (mode == SDF_GROUP_PERSISTENT && !grp->persist_ok && !grp->classes.empty())
    return fail(SDF_EUNSUPPORTED, "the persistent launch needs every member of width 128 or more, 512 at most");
  grp->mode = mode;
  return SDF_OK;
}

int sdf_group_collide_project(const sdf_group* grp, void* stream) {
  g_err.clear();
  if (!grp) return fail(SDF_EINVAL, "group is NULL");
  if (grp->classes.empty()) return SDF_OK;
  int prev = 0;
  (void)hipGetDevice(&prev);
  if (prev != grp->device) (void)hipSetDevice(grp->device);
  const hipError_t e = group_pass(grp, grp->classes[0].d_args, grp->args, (hipStream_t)stream);
  if (prev != grp->device) (void)hipSetDevice(prev);
  return e == hipSuccess ? SDF_OK : hip_fail(e, "kernel launch");
}

int sdf_net_autotune(sdf_net* net, int64_t n_sample, void* stream, int* variant) {
  g_err.clear();
  if (!net) return fail(SDF_EINVAL, "net is NULL");
  if (n_sample < 1 || n_sample > ((int64_t)1 << 26)) return fail(SDF_EINVAL, "n_sample must be in [1, 2^26]");
  if (!has_variant(net->W, net->prec)) {
    net->variant = 0;
    if (variant) *variant = 0;
    return SDF_OK;
  }
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(net->device);
  // points spread over [-1, 1]^3 (a fixed linear congruential sequence)
  std::vector<float> h((size_t)n_sample * 3);
  uint32_t st = 12345u;
  for (auto& v : h) {
    st = st * 1664525u + 1013904223u;
    v = (float)((st >> 8) * (2.0 / 16777216.0) - 1.0);
  }
  float* d = nullptr;
  if (hipMalloc(&d, h.size() * 4) != hipSuccess) {
    (void)hipSetDevice(prev);
    return fail(SDF_ENOMEM, "hipMalloc(autotune sample)");
  }
  const hipStream_t s = (hipStream_t)stream;
  float best = 0.0f;
  int pick = 0;
  for (int v = 0; v < 2; ++v) {
    if (hipMemcpy(d, h.data(), h.size() * 4, hipMemcpyHostToDevice) != hipSuccess) break;
    net->variant = v;
    const float ms = time_ms([&] { (void)run<MODE_PROJECT>(net, d, d, n_sample, 0.005f, nullptr, nullptr, nullptr, nullptr, s); }, s, 5);
    if (ms > 0.0f && (v == 0 || ms < best)) {
      best = ms;
      pick = v;
    }
  }
  net->variant = pick;
  (void)hipFree(d);
  (void)hipSetDevice(prev);
  if (variant) *variant = pick;
  return SDF_OK;
}

int sdf_net_set_tile_variant(sdf_net* net, int variant) {
  g_err.clear();
  if (!net) return fail(SDF_EINVAL, "net is NULL");
  if (variant != 0 && variant != 1) return fail(SDF_EINVAL, "variant must be 0 or 1");
  if (variant == 1 && !has_variant(net->W, net->prec))
    return fail(SDF_EUNSUPPORTED, "this network has one tile variant");
  net->variant = variant;
  return SDF_OK;
}

int sdf_group_autotune(sdf_group* grp, void* stream, int* mode_out) {
  g_err.clear();
  if (!grp) return fail(SDF_EINVAL, "group is NULL");
  if (grp->classes.empty()) return SDF_OK;
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(grp->device);
  const hipStream_t s = (hipStream_t)stream;
  // scratch copies of every vertex buffer, so the members' vertices are not moved
  int64_t total = 0;
  for (const auto& a : grp->args) total += a.n;
  float* scratch = nullptr;
  KArgs* d_tab = nullptr;
  const size_t tab_bytes = grp->args.size() * sizeof(KArgs);
  if (hipMalloc(&scratch, (size_t)total * 12 + 16) != hipSuccess || hipMalloc(&d_tab, tab_bytes) != hipSuccess) {
    if (scratch) (void)hipFree(scratch);
    (void)hipSetDevice(prev);
    return fail(SDF_ENOMEM, "hipMalloc(autotune scratch)");
  }
  std::vector<KArgs> tmp = grp->args;
  int64_t o = 0;
  for (auto& a : tmp) {
    a.pts_in = a.pts_out = scratch + 3 * o;
    o += a.n;
  }
  auto refill = [&] {  // the members' vertices, fresh for every timing
    int64_t q = 0;
    for (const auto& a : grp->args) {
      (void)hipMemcpyAsync(scratch + 3 * q, a.pts_in, (size_t)a.n * 12, hipMemcpyDeviceToDevice, s);
      q += a.n;
    }
  };
  hipError_t e = hipMemcpy(d_tab, tmp.data(), tab_bytes, hipMemcpyHostToDevice);
  // 1) tile variant per width class
  int off = 0;
  for (auto& c : grp->classes) {
    if (has_variant(c.W, grp->prec)) {
      float t[2];
      for (int v = 0; v < 2; ++v) {
        refill();
        t[v] = time_ms([&] { (void)launch_class(grp->prec, c, d_tab + off, c.d_start[v], v, s); }, s, 3);
      }
      c.var = (t[1] > 0.0f && t[1] < t[0]) ? 1 : 0;
    }
    off += c.n;
  }
  // 2) one launch per width class, one per network (networks keep their own
  // variant) or one persistent launch over everything (tile variant 0)
  std::vector<KArgs> ptmp(grp->n_persist);  // the persistent table over the scratch copies
  KArgs* d_ptab = nullptr;
  if (grp->persist_ok) {
    if (e == hipSuccess) e = hipMemcpy(ptmp.data(), grp->d_pargs, ptmp.size() * sizeof(KArgs), hipMemcpyDeviceToHost);
    for (auto& a : ptmp)
      for (size_t i = 0; i < grp->args.size(); ++i)
        if (grp->args[i].pts_in == a.pts_in) {
          a.pts_in = tmp[i].pts_in;
          a.pts_out = tmp[i].pts_out;
        }
    if (e == hipSuccess && hipMalloc(&d_ptab, ptmp.size() * sizeof(KArgs)) != hipSuccess) e = hipErrorOutOfMemory;
    if (e == hipSuccess) e = hipMemcpy(d_ptab, ptmp.data(), ptmp.size() * sizeof(KArgs), hipMemcpyHostToDevice);
  }
  float t[3] = {-1.0f, -1.0f, -1.0f};
  for (int m = 0; m < 3 && e == hipSuccess; ++m) {
    if (m == SDF_GROUP_PERSISTENT && !grp->persist_ok) continue;
    refill();
    if (m == SDF_GROUP_PERSISTENT)
      t[m] = time_ms([&] { (void)launch_persist(grp->prec, grp->cus, d_ptab, grp->d_pwidth, grp->d_pstart,
                                                grp->n_persist, grp->d_ctr, s); }, s, 3);
    else {
      grp->mode = m;
      t[m] = time_ms([&] { (void)group_pass(grp, d_tab, tmp, s); }, s, 3);
    }
  }
  int best = SDF_GROUP_PER_WIDTH;
  for (int m = 1; m < 3; ++m)
    if (t[m] > 0.0f && (t[best] <= 0.0f || t[m] < t[best])) best = m;
  grp->mode = best;
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(scratch);
  (void)hipFree(d_tab);
  if (d_ptab) (void)hipFree(d_ptab);
  (void)hipSetDevice(prev);
  if (mode_out) *mode_out = grp->mode;
  return e == hipSuccess ? SDF_OK : hip_fail(e, "autotune");
}

int sdf_verlet_step(float* pts, float* prev, int64_t n, float dt, const float* gravity, float damping,
                    void* stream) {
  g_err.clear();
  if (n < 0) return fail(SDF_EINVAL, "n < 0");
  if (!std::isfinite(dt) || !std::isfinite(damping) || !gravity) return fail(SDF_EINVAL, "bad dt, damping or gravity");
  for (int c = 0; c < 3; ++c)
    if (!std::isfinite(gravity[c])) return fail(SDF_EINVAL, "gravity must be finite");
  if (n == 0) return SDF_OK;
  if (!pts || !prev || !aligned4(pts) || !aligned4(prev)) return fail(SDF_EINVAL, "bad vertex buffers");
  if (pts == prev) return fail(SDF_EINVAL, "pts and prev must differ");
  const int64_t m = 3 * n;
  const double dt2 = (double)dt * (double)dt;
  const unsigned blocks = (unsigned)std::min<int64_t>((m + 255) / 256, 1 << 16);
  hipLaunchKernelGGL(verlet_kernel, dim3(blocks), dim3(256), 0, (hipStream_t)stream, pts, prev, m,
                     1.0f - damping, (float)(gravity[0] * dt2), (float)(gravity[1] * dt2), (float)(gravity[2] * dt2));
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? SDF_OK : hip_fail(e, "kernel launch");
}

}  // extern "C"
