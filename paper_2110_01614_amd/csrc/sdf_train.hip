// sdf_train.hip -- device kernels of one fitting step of the neural SDF
// (Sec. 3.1: an MLP regressed onto sampled signed distances with an L1
// loss, clamped to [-delta, delta]).
//
// A step over a batch runs, chunk by chunk:
//   pack:   the flat FP32 parameters -> FP32 MFMA fragment stream + small block
//           (the parameters change every step, so they are packed on device);
//   tile:   sdf_k32<W, MODE_TRAIN>: forward, dLoss/df, reverse sweep; writes
//           h_l and e_l = dLoss/dz_l of every point of the chunk;
//   wgrad:  grad += sum_p e_l(p) [h_{l-1}(p), x(p), 1]^T for every layer and
//           the output layer, on v_mfma_f32_16x16x4_f32;
//   loss:   loss += sum_p |clamp(f_p) - clamp(s_p)| / n.
// Each output element is owned by one thread of one workgroup and chunks run
// in stream order, so the result does not depend on scheduling.
#include "sdf_device.hpp"

namespace sdfc {

// params -> FP32 fragment stream (same order as the host packer: forward
// layers 2..L then reverse layers L..2; fragment (mt, m), lane 16g+row,
// element i holds A[16mt + row][16m + 4g + i]) and the small FP32 block.
__global__ void __launch_bounds__(256) pack_fp32_kernel(TrainNet t, const float* __restrict__ P,
                                                        float* __restrict__ stream,
                                                        float* __restrict__ small) {
  const int W = t.W, L = t.L, MT = W / 16;
  const int64_t per_layer = (int64_t)MT * MT * 64 * 4;
  const int64_t total = 2 * (int64_t)(L - 1) * per_layer;
  const SmallLayout SL{W};
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total + W;
       idx += (int64_t)gridDim.x * blockDim.x) {
    if (idx < total) {
      const int64_t layer_id = idx / per_layer;
      int64_t r = idx % per_layer;
      const int i = (int)(r & 3);
      const int lane = (int)((r >> 2) & 63);
      r >>= 8;
      const int m = (int)(r % MT), mt = (int)(r / MT);
      const int pass = (int)(layer_id / (L - 1)), s = (int)(layer_id % (L - 1));
      const int l = pass == 0 ? 2 + s : L - s;
      const int row = 16 * mt + (lane & 15), col = 16 * m + 4 * (lane >> 4) + i;
      const int K = t.K(l);
      const float* Wl = P + t.offW[l];
      stream[idx] = pass == 0 ? Wl[(int64_t)row * K + col] : Wl[(int64_t)col * K + row];
    } else {
      const int j = (int)(idx - total);
      const float kap = t.kappa;
      const float* w1 = P + t.offW[1] + 3 * j;
      for (int c = 0; c < 3; ++c) {
        small[SL.l1() + 4 * j + c] = kap * w1[c];
        small[SL.l1g() + 4 * j + c] = w1[c];
        float sf = 0.0f, sg = 0.0f;
        if (t.skip) {
          const float ws = P[t.offW[t.skip] + (int64_t)j * t.K(t.skip) + W + c];
          sf = kap * ws;
          sg = ws;
        }
        small[SL.skf() + 4 * j + c] = sf;
        small[SL.skg() + 4 * j + c] = sg;
      }
      small[SL.l1() + 4 * j + 3] = kap * P[t.offb[1] + j];
      small[SL.l1g() + 4 * j + 3] = 0.0f;
      small[SL.skf() + 4 * j + 3] = 0.0f;
      small[SL.skg() + 4 * j + 3] = 0.0f;
      small[SL.wof() + j] = P[t.offo + j] / kap;
      small[SL.wob() + j] = P[t.offo + j];
      for (int l = 2; l <= kLMax; ++l) small[SL.bias(l) + j] = l <= L ? kap * P[t.offb[l] + j] : 0.0f;
    }
  }
}

__global__ void __launch_bounds__(256) fill_kernel(float* __restrict__ p, int64_t n, float v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// loss += sum of the chunk's per-point terms: one workgroup of 1024
// threads; each thread adds its 16-byte groups of terms (four loads in
// flight per step), thread 0 the n % 4 last terms, then a tree over the
// threads.  The order is fixed.
constexpr int kLossThreads = 1024;
__global__ void __launch_bounds__(kLossThreads) loss_reduce_kernel(const float* __restrict__ terms, int64_t n,
                                                                   float* __restrict__ loss) {
  __shared__ float part[kLossThreads];
  const int64_t n4 = n / 4;
  const float4* t4 = reinterpret_cast<const float4*>(terms);  // the terms buffer is 256-byte aligned
  float s = 0.0f;
  for (int64_t i = threadIdx.x; i < n4; i += 4 * kLossThreads) {
    float4 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t j = i + (int64_t)u * kLossThreads;
      v[u] = j < n4 ? t4[j] : float4{0.0f, 0.0f, 0.0f, 0.0f};
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) s += (v[u].x + v[u].y) + (v[u].z + v[u].w);
  }
  if (threadIdx.x == 0)
    for (int64_t j = 4 * n4; j < n; ++j) s += terms[j];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int w = kLossThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[0] += part[0];
}

// Work item `item` of the weight-gradient contraction with BS x BS output
// blocks: hidden layer l (1..L) or the output layer (l = L + 1), a block of
// BS output rows and a block of BS input columns (or the 16-wide tail block:
// x, y, z, 1, zeros).
struct WItem {
  int l, rb, cb;
};

template <int BS>
__device__ __forceinline__ WItem wgrad_item(const TrainNet& t, int item) {
  const int W = t.W, L = t.L;
  const int RB = W / BS, CB = W / BS + 1;  // row blocks; column blocks + the 16-wide tail
  if (item < RB) return {1, item, CB - 1};  // layer 1: tail columns only
  item -= RB;
  if (item < (L - 1) * RB * CB) return {2 + item / (RB * CB), (item / CB) % RB, item % CB};
  item -= (L - 1) * RB * CB;
  return {L + 1, 0, item};
}

// Flat-parameter index of the gradient of output row j, input column k of
// layer l (k < W: hidden input; W..W+2: x, y, z; W+3: bias), or -1.
__device__ __forceinline__ int64_t wgrad_dst(const TrainNet& t, int l, int j, int k) {
  const int W = t.W, L = t.L;
  if (l == L + 1) {  // output layer: one real row
    if (j != 0) return -1;
    return (k < W) ? t.offo + k : (k == W + 3 ? t.offo + W : -1);
  }
  if (k < W) return t.offW[l] + (int64_t)j * t.K(l) + k;  // hidden input columns (l >= 2)
  if (k < W + 3) {
    const int c = k - W;
    if (l == 1) return t.offW[1] + 3 * j + c;
    if (l == t.skip) return t.offW[l] + (int64_t)j * t.K(l) + W + c;
    return -1;
  }
  if (k == W + 3) return t.offb[l] + j;
  return -1;
}

// sum_p E[p][rows] (x) H[p][cols] for one work item over one slice of the
// chunk's points.  Hidden layer l (1..L): E = e_l [n][W], H = H_{l-1}
// [n][W+16] whose columns are h_{l-1} (W), x, y, z, 1, zeros.  Output layer
// (l = L+1): E = dLoss/df [n][16] (row 0), H = H_L.  Columns map to dW_l
// (hidden and skip x-columns), db_l (the "1" column), dw_o and db_o.
// Workgroup b takes item b % items and point slice b / items of nsplit
// slices of whole 16-point tiles.  Each tile of the block's E rows and H
// columns is staged in LDS with 16-byte loads (read from global once per
// workgroup, the next tile's loads in flight while the current one is
// contracted); wave w contracts a 32 x 64 part of the BS x BS block on
// v_mfma_f32_16x16x4_f32 (BS = 128: 8 waves, so every staged byte feeds
// twice the MFMAs of a 64 x 64 block).  nsplit == 1: grad += the sum
// directly (one owner per element); otherwise the block is written to
// part[slice][item][BS][BS] and wgrad_reduce_kernel adds the slices in a
// fixed order.
constexpr int kWgP = 16;  // points per staged tile
template <int BS>
__global__ void __launch_bounds__(BS * BS / 32) wgrad_kernel(TrainNet t, const float* __restrict__ E,
                                                             const float* __restrict__ H,
                                                             const float* __restrict__ U, int64_t n, int items,
                                                             int nsplit, float* __restrict__ part,
                                                             float* __restrict__ grad) {
  constexpr int NT = BS * BS / 32;        // threads: (BS / 32) x (BS / 64) waves
  constexpr int WR = BS / 32;             // waves along the rows
  constexpr int S = BS + 16;              // LDS row stride in floats: the four point rows one MFMA reads start 16 banks apart
  constexpr int NLD = (BS / 4 * kWgP + NT - 1) / NT;  // float4 loads per thread per operand
  __shared__ __attribute__((aligned(16))) float sE[2][kWgP * S];
  __shared__ __attribute__((aligned(16))) float sH[2][kWgP * S];
  const int W = t.W, L = t.L;
  const int item = blockIdx.x % items, slice = blockIdx.x / items;
  const WItem wi = wgrad_item<BS>(t, item);
  const int l = wi.l, CB = W / BS + 1;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave % WR, wc = wave / WR;  // this wave: rows 32 wr.., columns 64 wc.. of the block
  const int g = lane >> 4, c16 = lane & 15;
  const bool out_layer = (l == L + 1);
  const bool tail = (wi.cb == CB - 1);
  const int col0 = tail ? W : BS * wi.cb;
  const float* Eb = out_layer ? U : E + (size_t)(l - 1) * n * W;
  const int es = out_layer ? 16 : W;
  const int er0 = out_layer ? 0 : BS * wi.rb;  // first staged E column
  const int ew4 = out_layer ? 4 : BS / 4;      // staged E columns / 4
  const float* Hb = H + (size_t)(l - 1) * n * (W + 16);
  const int hs = W + 16;
  const int hw4 = tail ? 4 : BS / 4;           // staged H columns / 4
  // only the staged rows and columns exist: the output layer has 16 rows
  // (row 0 real), a tail block 16 columns (all waves still stage)
  const int nrt = out_layer ? 1 : 2, nct = tail ? 1 : 4;
  const bool active = (wr == 0 || !out_layer) && (wc == 0 || !tail);
  const int64_t tiles = (n + kWgP - 1) / kWgP;
  const int64_t t_lo = tiles * slice / nsplit, t_hi = tiles * (slice + 1) / nsplit;
  const int qE = ew4 * kWgP, qH = hw4 * kWgP;  // float4s of a staged tile
  float4 rE[NLD], rH[NLD];
  auto load = [&](int64_t tile) {
    const int64_t p0 = tile * kWgP;
#pragma unroll
    for (int i = 0; i < NLD; ++i) {
      const int q = tid + NT * i;
      if (q < qE) {
        const int64_t p = p0 + q / ew4;
        rE[i] = p < n ? *reinterpret_cast<const float4*>(Eb + p * es + er0 + 4 * (q % ew4))
                      : float4{0.0f, 0.0f, 0.0f, 0.0f};
      }
      if (q < qH) {
        const int64_t p = p0 + q / hw4;
        rH[i] = p < n ? *reinterpret_cast<const float4*>(Hb + p * hs + col0 + 4 * (q % hw4))
                      : float4{0.0f, 0.0f, 0.0f, 0.0f};
      }
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int i = 0; i < NLD; ++i) {
      const int q = tid + NT * i;
      if (q < qE) *reinterpret_cast<float4*>(&sE[buf][(q / ew4) * S + 4 * (q % ew4)]) = rE[i];
      if (q < qH) *reinterpret_cast<float4*>(&sH[buf][(q / hw4) * S + 4 * (q % hw4)]) = rH[i];
    }
  };
  f32x4 acc[2][4] = {};
  if (t_lo < t_hi) load(t_lo);
  for (int64_t tt = t_lo; tt < t_hi; ++tt) {
    const int buf = (int)((tt - t_lo) & 1);
    store(buf);  // buffer buf was last read two tiles ago, before the previous barrier
    __syncthreads();
    if (tt + 1 < t_hi) load(tt + 1);
    if (active) {
      __builtin_amdgcn_s_setprio(1);  // MFMAs ahead of the other waves' staging (about 1 % of a step)
      const float* e = sE[buf];
      const float* h = sH[buf];
#pragma unroll
      for (int k = 0; k < kWgP; k += 4) {
        const float* er = e + (k + g) * S + 32 * wr + c16;
        const float* hr = h + (k + g) * S + 64 * wc + c16;
#pragma unroll
        for (int rt = 0; rt < 2; ++rt) {
          if (rt < nrt) {
            const float a = er[16 * rt];
#pragma unroll
            for (int ct = 0; ct < 4; ++ct)
              if (ct < nct) acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, hr[16 * ct], acc[rt][ct], 0, 0, 0);
          }
        }
      }
      __builtin_amdgcn_s_setprio(0);
    }
  }
  if (!active) return;
  // acc[rt][ct][i] = sum_p E[p][er0 + 32 wr + 16 rt + 4g + i] H[p][col0 + 64 wc + 16 ct + c16]
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
      if (rt >= nrt || ct >= nct) continue;  // (constant indices: acc stays in registers)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float v = acc[rt][ct][i];
        const int r = 32 * wr + 16 * rt + 4 * g + i, c = 64 * wc + 16 * ct + c16;
        if (nsplit > 1) {
          part[(((size_t)slice * items + item) * BS + r) * BS + c] = v;
        } else {
          const int64_t dst = wgrad_dst(t, l, (out_layer ? 0 : BS * wi.rb) + r, col0 + c);
          if (dst >= 0) grad[dst] += v;
        }
      }
    }
}

// grad += sum over the nsplit slices (in slice order) of every work item's
// BS x BS block; one thread per block element.
template <int BS>
__global__ void __launch_bounds__(256) wgrad_reduce_kernel(TrainNet t, const float* __restrict__ part,
                                                           int items, int nsplit, float* __restrict__ grad) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)items * BS * BS) return;
  const int item = (int)(idx / (BS * BS)), r = (int)((idx / BS) % BS), c = (int)(idx % BS);
  const WItem wi = wgrad_item<BS>(t, item);
  const int W = t.W, CB = W / BS + 1;
  const bool out_layer = (wi.l == t.L + 1), tail = (wi.cb == CB - 1);
  if ((tail && c >= 16) || (out_layer && r >= 16)) return;  // never written
  const int j = out_layer ? r : BS * wi.rb + r;
  const int64_t dst = wgrad_dst(t, wi.l, j, (tail ? W : BS * wi.cb) + c);
  if (dst < 0) return;
  float s = 0.0f;
  for (int q = 0; q < nsplit; ++q) s += part[(((size_t)q * items + item) * BS + r) * BS + c];
  grad[dst] += s;
}

template __global__ void wgrad_kernel<64>(TrainNet, const float*, const float*, const float*, int64_t, int, int,
                                          float*, float*);
template __global__ void wgrad_kernel<128>(TrainNet, const float*, const float*, const float*, int64_t, int, int,
                                           float*, float*);
template __global__ void wgrad_reduce_kernel<64>(TrainNet, const float*, int, int, float*);
template __global__ void wgrad_reduce_kernel<128>(TrainNet, const float*, int, int, float*);

}  // namespace sdfc
