// sdf_k16.hip -- fused neural-SDF query / gradient / collision kernel with
// 16-bit (BF16 or FP16) MFMA operands and FP32 accumulation, for gfx950.
//
// One workgroup = 4 wave64 = 64 points; each wave owns 16 points for the whole
// pass.  Per hidden layer l >= 2 the wave computes the 16-point column block
// of z_l = W_l r_{l-1} with v_mfma_f32_16x16x32_{bf16,f16}: A = a weight
// fragment read from LDS, B = the previous layer's activations, which never
// leave registers (Sec. 3.1, Eq. 1).  The input gradient is the reverse sweep
// of Sec. 3.2 over the same weights transposed.  Every r_l (16-bit) stays in
// registers for that sweep (the "stack"); each sigmoid is recovered as
// 1 - 2^{-r}.  Layer 1 (K = 3), the skip x-columns, the output layer, the
// normal (Eq. 2) and the move to the contact point (Eq. 3) are FP32 VALU.
//
// Weights stream through a 4-slot LDS ring in 32 KB chunks with direct
// global->LDS copies (see sdf_device.hpp); two chunks stay in flight while
// the workgroup computes on the third.
#include "sdf_device.hpp"

namespace sdfc {

template <int PREC>
__device__ __forceinline__ void put4(u32x4& v, int half, const float r[4]) {
  v[2 * half] = pack2<PREC>(r[0], r[1]);
  v[2 * half + 1] = pack2<PREC>(r[2], r[3]);
}

template <int PREC>
__device__ __forceinline__ void get4(const u32x4& v, int half, float r[4]) {
  unpack2<PREC>(v[2 * half], r[0], r[1]);
  unpack2<PREC>(v[2 * half + 1], r[2], r[3]);
}

template <int W, int PREC, int MODE>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(1, 1)))
sdf_k16(const KArgs a) {
  using G = Geo<W, false>;
  constexpr SmallLayout SL{W};
  constexpr int KB = G::KB, MT = G::MT, CH_MT = G::CH_MT, CPL = G::CPL;
  static_assert(kNBuf == 4, "chunk_acquire assumes a 4-slot ring");

  __shared__ __attribute__((aligned(1024))) unsigned char ring[kNBuf * G::CHUNK];
  __shared__ __attribute__((aligned(16))) float sm[SL.floats()];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int g = lane >> 4;
  const int64_t p = (int64_t)blockIdx.x * kPtsPerBlock + wave * kPtsPerWave + (lane & 15);
  const bool valid = p < a.n;
  const int L = a.L, skip = a.skip, nch = a.nch;

  // ---- point, small FP32 weights ----
  float x0 = 0.0f, x1 = 0.0f, x2 = 0.0f;
  if (valid) {
    x0 = a.pts_in[3 * p];
    x1 = a.pts_in[3 * p + 1];
    x2 = a.pts_in[3 * p + 2];
  }
  for (int i = tid; i < SL.floats() / 4; i += kBlock)
    reinterpret_cast<f32x4*>(sm)[i] = reinterpret_cast<const f32x4*>(a.small)[i];
  __syncthreads();

  const unsigned ring0 = lds_u32(ring);
  for (int c = 0; c < kNBuf - 1; ++c)
    if (c < nch) issue_chunk<G>(a.stream, c, ring0, wave, lane);

  // ---- layer 1: y = kappa (W1 x + b1), K = 3, FP32 VALU ----
  u32x4 stk[kLMax][KB];  // stk[l] = r_l in B-operand order, l = 1..L-1
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) {
    float r[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const f32x4 w = *reinterpret_cast<const f32x4*>(&sm[SL.l1() + 4 * (16 * mt + 4 * g + i)]);
      r[i] = softplus2(__builtin_fmaf(w.x, x0, __builtin_fmaf(w.y, x1, __builtin_fmaf(w.z, x2, w.w))));
    }
    put4<PREC>(stk[1][mt >> 1], mt & 1, r);
  }

  float fpart = 0.0f, gx0 = 0.0f, gx1 = 0.0f, gx2 = 0.0f;
  u32x4 D0[KB], D1[KB];  // d_l (scaled) in B-operand order; d_l lives in D[l & 1]
  int gc = 0;

  // ---- hidden layers 2..L, forward ----
#pragma unroll
  for (int l = 2; l <= kLMax; ++l) {
    if (l > L) break;
    const bool last = (l == L);
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
      chunk_acquire<G>(gc, nch, a.stream, ring0, wave, lane);
      const unsigned char* buf = ring + (gc % kNBuf) * G::CHUNK;
#pragma unroll
      for (int mm = 0; mm < CH_MT; mm += 2) {
        const int mt = c * CH_MT + mm;
        f32x4 acc[2];
#pragma unroll
        for (int h = 0; h < 2; ++h)
          acc[h] = *reinterpret_cast<const f32x4*>(&sm[SL.bias(l) + 16 * (mt + h) + 4 * g]);
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const u32x4 A = *reinterpret_cast<const u32x4*>(buf + ((mm + h) * KB + kb) * kFrag + lane * 16);
            acc[h] = mfma16<PREC>(A, stk[l - 1][kb], acc[h]);
          }
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int m = mt + h;
          if (l == skip) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const f32x4 w = *reinterpret_cast<const f32x4*>(&sm[SL.skf() + 4 * (16 * m + 4 * g + i)]);
              acc[h][i] = __builtin_fmaf(w.x, x0, __builtin_fmaf(w.y, x1, __builtin_fmaf(w.z, x2, acc[h][i])));
            }
          }
          float r[4];
#pragma unroll
          for (int i = 0; i < 4; ++i) r[i] = softplus2(acc[h][i]);
          if (!last) {
            put4<PREC>(stk[l][m >> 1], m & 1, r);
          } else {
            const f32x4 wf = *reinterpret_cast<const f32x4*>(&sm[SL.wof() + 16 * m + 4 * g]);
#pragma unroll
            for (int i = 0; i < 4; ++i) fpart = __builtin_fmaf(wf[i], r[i], fpart);
            if constexpr (MODE != MODE_QUERY) {
              const f32x4 wb = *reinterpret_cast<const f32x4*>(&sm[SL.wob() + 16 * m + 4 * g]);
              float d[4];
#pragma unroll
              for (int i = 0; i < 4; ++i)  // d_L = w_o * sigmoid = w_o (1 - 2^-r)
                d[i] = __builtin_fmaf(-wb[i], __builtin_amdgcn_exp2f(-r[i]), wb[i]);
              if (l == skip) {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                  const f32x4 w = *reinterpret_cast<const f32x4*>(&sm[SL.skg() + 4 * (16 * m + 4 * g + i)]);
                  gx0 = __builtin_fmaf(w.x, d[i], gx0);
                  gx1 = __builtin_fmaf(w.y, d[i], gx1);
                  gx2 = __builtin_fmaf(w.z, d[i], gx2);
                }
              }
              put4<PREC>((l & 1) ? D1[m >> 1] : D0[m >> 1], m & 1, d);
            }
          }
        }
      }
      ++gc;
    }
  }

  // ---- reverse sweep: layers L..2 over W_l^T ----
  if constexpr (MODE != MODE_QUERY) {
#pragma unroll
    for (int l = kLMax; l >= 2; --l) {
      if (l > L) continue;
#pragma unroll
      for (int c = 0; c < CPL; ++c) {
        chunk_acquire<G>(gc, nch, a.stream, ring0, wave, lane);
        const unsigned char* buf = ring + (gc % kNBuf) * G::CHUNK;
#pragma unroll
        for (int mm = 0; mm < CH_MT; mm += 2) {
          const int mt = c * CH_MT + mm;
          f32x4 acc[2] = {{0.0f, 0.0f, 0.0f, 0.0f}, {0.0f, 0.0f, 0.0f, 0.0f}};
#pragma unroll
          for (int kb = 0; kb < KB; ++kb) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
              const u32x4 A = *reinterpret_cast<const u32x4*>(buf + ((mm + h) * KB + kb) * kFrag + lane * 16);
              acc[h] = mfma16<PREC>(A, (l & 1) ? D1[kb] : D0[kb], acc[h]);
            }
          }
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int m = mt + h;
            float r[4], d[4];
            get4<PREC>(stk[l - 1][m >> 1], m & 1, r);
#pragma unroll
            for (int i = 0; i < 4; ++i)  // d_{l-1} = g (1 - 2^-r_{l-1})
              d[i] = __builtin_fmaf(-acc[h][i], __builtin_amdgcn_exp2f(-r[i]), acc[h][i]);
            if (l - 1 == skip || l == 2) {
              const int off = (l == 2) ? SL.l1g() : SL.skg();
#pragma unroll
              for (int i = 0; i < 4; ++i) {
                const f32x4 w = *reinterpret_cast<const f32x4*>(&sm[off + 4 * (16 * m + 4 * g + i)]);
                gx0 = __builtin_fmaf(w.x, d[i], gx0);
                gx1 = __builtin_fmaf(w.y, d[i], gx1);
                gx2 = __builtin_fmaf(w.z, d[i], gx2);
              }
            }
            if (l > 2) put4<PREC>((l & 1) ? D0[m >> 1] : D1[m >> 1], m & 1, d);
          }
        }
        ++gc;
      }
    }
  }

  const float f = sum_lane_groups(fpart) + a.bo;
  if constexpr (MODE != MODE_QUERY) {
    gx0 = sum_lane_groups(gx0);
    gx1 = sum_lane_groups(gx1);
    gx2 = sum_lane_groups(gx2);
  }
  store_outputs<MODE>(a, p, valid && g == 0, f, gx0, gx1, gx2, x0, x1, x2);
}

#define SDF_K16_INST(W, PREC, MODE) \
  template __global__ void sdf_k16<W, PREC, MODE>(const KArgs);
#define SDF_K16_MODES(W, PREC) \
  SDF_K16_INST(W, PREC, MODE_QUERY) SDF_K16_INST(W, PREC, MODE_GRAD) SDF_K16_INST(W, PREC, MODE_PROJECT)
SDF_K16_MODES(64, PREC_BF16)
SDF_K16_MODES(128, PREC_BF16)
SDF_K16_MODES(256, PREC_BF16)
SDF_K16_MODES(64, PREC_FP16)
SDF_K16_MODES(128, PREC_FP16)
SDF_K16_MODES(256, PREC_FP16)

}  // namespace sdfc
