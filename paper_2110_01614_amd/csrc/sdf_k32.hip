// sdf_k32.hip -- fused neural-SDF query / gradient / collision kernel with
// FP32 MFMA operands (v_mfma_f32_16x16x4_f32), for gfx950.
//
// Same structure as the 16-bit kernel: a workgroup of 4 wave64 handles 64
// points, 16 per wave; weights stream through a 4-slot LDS ring; activations
// stay in registers between layers (an accumulator register of M-tile m is
// directly the B operand of K-block (m, i) of the next layer).  FP32 r_l for
// 8 layers of 256 units do not fit next to everything else, so the forward
// pass stores the sigmoids s_l = sigmoid(beta z_l) of layers 1..L-1 in a
// per-workgroup scratch area (one slot per resident workgroup, reused tile
// after tile) and the reverse sweep (Sec. 3.2) reads them back.  The grid is
// persistent: workgroup b processes tiles b, b + gridDim.x, ...
//
// MODE_TRAIN (fitting, Sec. 3.1) runs the same two sweeps for the clamped-L1
// loss: the reverse sweep is seeded with dLoss/df instead of 1, and every
// layer's activations h_l and errors dLoss/dz_l are written to a workspace
// from which the weight-gradient kernel (sdf_train.hip) forms sum_p e h^T.
#include "sdf_device.hpp"

namespace sdfc {

// sigmoid(beta z) from y = kappa z: 1/(1 + 2^-y) (y >= 0) or 2^y/(1 + 2^y).
__device__ __forceinline__ void softplus_sigmoid(float y, float& r, float& s) {
  const float e = __builtin_amdgcn_exp2f(-__builtin_fabsf(y));
  const float t = 1.0f + e;
  r = __builtin_fmaxf(y, 0.0f) + __builtin_amdgcn_logf(t);
  const float q = __builtin_amdgcn_rcpf(t);
  s = (y >= 0.0f) ? q : e * q;
}

// Workspace row pointers of point p (training): H_l row and E_l row.
template <int W>
__device__ __forceinline__ float* hrow(const KArgs& a, int l, int64_t p) {
  return a.ws_H + ((size_t)l * a.n + p) * (W + 16);
}
template <int W>
__device__ __forceinline__ float* erow(const KArgs& a, int l, int64_t p) {
  return a.ws_E + ((size_t)(l - 1) * a.n + p) * W;
}

template <int W, int MODE>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(1, 1)))
sdf_k32(const KArgs a) {
  constexpr bool TRAIN = MODE == MODE_TRAIN;
  using G = Geo<W, true>;
  constexpr SmallLayout SL{W};
  constexpr int MT = G::MT, KB = G::KB, CH_MT = G::CH_MT, CPL = G::CPL;
  static_assert(kNBuf == 4, "chunk_acquire assumes a 4-slot ring");

  __shared__ __attribute__((aligned(1024))) unsigned char ring[kNBuf * G::CHUNK];
  __shared__ __attribute__((aligned(16))) float sm[SL.floats()];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int g = lane >> 4;
  const int L = a.L, skip = a.skip, nch = a.nch;
  const unsigned ring0 = lds_u32(ring);

  for (int i = tid; i < SL.floats() / 4; i += kBlock)
    reinterpret_cast<f32x4*>(sm)[i] = reinterpret_cast<const f32x4*>(a.small)[i];

  // sigma stack of this workgroup: [layer 1..kLMax-1][wave][M-tile][lane] float4
  f32x4* sstk = reinterpret_cast<f32x4*>(a.scratch) +
                (size_t)blockIdx.x * (kLMax - 1) * 4 * MT * 64 + wave * MT * 64 + lane;
  constexpr size_t kLayerStride = (size_t)4 * MT * 64;

  for (int tile = blockIdx.x; tile < a.ntiles; tile += gridDim.x) {
    const int64_t p = (int64_t)tile * kPtsPerBlock + wave * kPtsPerWave + (lane & 15);
    const bool valid = p < a.n;
    float w0 = 0.0f, w1 = 0.0f, w2 = 0.0f;  // as loaded (world frame)
    if (valid) {
      w0 = a.pts_in[3 * p];
      w1 = a.pts_in[3 * p + 1];
      w2 = a.pts_in[3 * p + 2];
    }
    float x0 = w0, x1 = w1, x2 = w2;  // in the network's frame
    to_local(a, x0, x1, x2);
    __syncthreads();  // small weights visible; previous tile done with the ring
    for (int c = 0; c < kNBuf - 1; ++c)
      if (c < nch) issue_chunk<G>(a.stream, c, ring0, wave, lane);

    f32x4 Rin[MT], Rout[MT];  // r_{l-1} (B operands) and r_l being produced
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      f32x4 s4;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const f32x4 w = *reinterpret_cast<const f32x4*>(&sm[SL.l1() + 4 * (16 * mt + 4 * g + i)]);
        float r, sg;
        softplus_sigmoid(__builtin_fmaf(w.x, x0, __builtin_fmaf(w.y, x1, __builtin_fmaf(w.z, x2, w.w))), r, sg);
        Rin[mt][i] = r;
        s4[i] = sg;
      }
      if constexpr (MODE != MODE_QUERY) sstk[mt * 64] = s4;
      if constexpr (TRAIN)
        if (valid) *reinterpret_cast<f32x4*>(hrow<W>(a, 1, p) + 16 * mt + 4 * g) = Rin[mt] * a.inv_kappa;
    }
    if constexpr (TRAIN) {
      if (valid && g == 0) {  // h_0 slot: x, y, z, 1 in the extra columns of every H row
#pragma unroll
        for (int l = 0; l <= kLMax; ++l) {
          if (l > L) break;
          float* row = hrow<W>(a, l, p) + W;
          *reinterpret_cast<f32x4*>(row) = f32x4{x0, x1, x2, 1.0f};
#pragma unroll
          for (int c = 4; c < 16; c += 4) *reinterpret_cast<f32x4*>(row + c) = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
        }
      }
    }

    float fpart = 0.0f, gx0 = 0.0f, gx1 = 0.0f, gx2 = 0.0f;
    f32x4 Din[MT], Dout[MT];  // d_l (B operands) and d_{l-1} being produced
    int gc = 0;

    for (int l = 2; l <= L; ++l) {
      const bool last = (l == L);
      const bool at_skip = (l == skip);
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
          // queries: raised wave priority while issuing the MFMAs, so they go
          // ahead of the other waves' epilogues (about 4 %; the fitting mode,
          // which also writes every activation out, is about 1 % slower with it)
          if constexpr (!TRAIN) __builtin_amdgcn_s_setprio(1);
#pragma unroll
          for (int m = 0; m < KB; ++m) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
              const f32x4 A = *reinterpret_cast<const f32x4*>(buf + ((mm + h) * KB + m) * kFrag + lane * 16);
#pragma unroll
              for (int i = 0; i < 4; ++i)
                acc[h] = __builtin_amdgcn_mfma_f32_16x16x4f32(A[i], Rin[m][i], acc[h], 0, 0, 0);
            }
          }
          if constexpr (!TRAIN) __builtin_amdgcn_s_setprio(0);
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int m = mt + h;
            if (at_skip) {
#pragma unroll
              for (int i = 0; i < 4; ++i) {
                const f32x4 w = *reinterpret_cast<const f32x4*>(&sm[SL.skf() + 4 * (16 * m + 4 * g + i)]);
                acc[h][i] = __builtin_fmaf(w.x, x0, __builtin_fmaf(w.y, x1, __builtin_fmaf(w.z, x2, acc[h][i])));
              }
            }
            f32x4 r4, s4;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              float r, sg;
              softplus_sigmoid(acc[h][i], r, sg);
              r4[i] = r;
              s4[i] = sg;
            }
            Rout[m] = r4;
            if constexpr (TRAIN)
              if (valid) *reinterpret_cast<f32x4*>(hrow<W>(a, l, p) + 16 * m + 4 * g) = r4 * a.inv_kappa;
            if (!last) {
              if constexpr (MODE != MODE_QUERY) sstk[(l - 1) * kLayerStride + m * 64] = s4;
            } else {
              const f32x4 wf = *reinterpret_cast<const f32x4*>(&sm[SL.wof() + 16 * m + 4 * g]);
#pragma unroll
              for (int i = 0; i < 4; ++i) fpart = __builtin_fmaf(wf[i], r4[i], fpart);
              if constexpr (MODE != MODE_QUERY) {
                const f32x4 wb = *reinterpret_cast<const f32x4*>(&sm[SL.wob() + 16 * m + 4 * g]);
                const f32x4 d = wb * s4;
                if (!TRAIN && at_skip) {
#pragma unroll
                  for (int i = 0; i < 4; ++i) {
                    const f32x4 w = *reinterpret_cast<const f32x4*>(&sm[SL.skg() + 4 * (16 * m + 4 * g + i)]);
                    gx0 = __builtin_fmaf(w.x, d[i], gx0);
                    gx1 = __builtin_fmaf(w.y, d[i], gx1);
                    gx2 = __builtin_fmaf(w.z, d[i], gx2);
                  }
                }
                Din[m] = d;
              }
            }
          }
        }
        ++gc;
      }
#pragma unroll
      for (int m = 0; m < MT; ++m) Rin[m] = Rout[m];
    }

    float f = sum_lane_groups(fpart) + (TRAIN ? a.bo_dev[0] : a.bo);
    if constexpr (TRAIN) {
      // clamped L1: dLoss/df = sign(clamp(f) - clamp(s)) [-delta <= f <= delta] / n
      float u = 0.0f, lp = 0.0f;
      if (valid) {
        const float s = a.target[p];
        const float cf = __builtin_fminf(__builtin_fmaxf(f, -a.delta), a.delta);
        const float cs = __builtin_fminf(__builtin_fmaxf(s, -a.delta), a.delta);
        const float r = cf - cs;
        lp = __builtin_fabsf(r) * a.inv_n;
        if (f >= -a.delta && f <= a.delta) u = (r > 0.0f ? a.inv_n : (r < 0.0f ? -a.inv_n : 0.0f));
        if (g == 0) {
          a.ws_loss[p] = lp;
          float* urow = a.ws_U + 16 * p;
          *reinterpret_cast<f32x4*>(urow) = f32x4{u, 0.0f, 0.0f, 0.0f};
#pragma unroll
          for (int c = 4; c < 16; c += 4) *reinterpret_cast<f32x4*>(urow + c) = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
        }
      }
#pragma unroll
      for (int m = 0; m < MT; ++m) Din[m] = Din[m] * u;  // seed d_L = u w_o sigma_L
    }

    if constexpr (MODE != MODE_QUERY) {
      for (int l = L; l >= 2; --l) {
        const bool to_skip = (l - 1 == skip), to_input = (l == 2);
        if constexpr (TRAIN)
          if (valid)
#pragma unroll
            for (int m = 0; m < MT; ++m) *reinterpret_cast<f32x4*>(erow<W>(a, l, p) + 16 * m + 4 * g) = Din[m];
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
          chunk_acquire<G>(gc, nch, a.stream, ring0, wave, lane);
          const unsigned char* buf = ring + (gc % kNBuf) * G::CHUNK;
#pragma unroll
          for (int mm = 0; mm < CH_MT; mm += 2) {
            const int mt = c * CH_MT + mm;
            f32x4 acc[2] = {{0.0f, 0.0f, 0.0f, 0.0f}, {0.0f, 0.0f, 0.0f, 0.0f}};
            f32x4 s[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) s[h] = sstk[(l - 2) * kLayerStride + (mt + h) * 64];
            if constexpr (!TRAIN) __builtin_amdgcn_s_setprio(1);
#pragma unroll
            for (int m = 0; m < KB; ++m) {
#pragma unroll
              for (int h = 0; h < 2; ++h) {
                const f32x4 A = *reinterpret_cast<const f32x4*>(buf + ((mm + h) * KB + m) * kFrag + lane * 16);
#pragma unroll
                for (int i = 0; i < 4; ++i)
                  acc[h] = __builtin_amdgcn_mfma_f32_16x16x4f32(A[i], Din[m][i], acc[h], 0, 0, 0);
              }
            }
            if constexpr (!TRAIN) __builtin_amdgcn_s_setprio(0);
#pragma unroll
            for (int h = 0; h < 2; ++h) {
              const int m = mt + h;
              const f32x4 d = acc[h] * s[h];
              if (!TRAIN && (to_skip || to_input)) {
                const int off = to_input ? SL.l1g() : SL.skg();
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                  const f32x4 w = *reinterpret_cast<const f32x4*>(&sm[off + 4 * (16 * m + 4 * g + i)]);
                  gx0 = __builtin_fmaf(w.x, d[i], gx0);
                  gx1 = __builtin_fmaf(w.y, d[i], gx1);
                  gx2 = __builtin_fmaf(w.z, d[i], gx2);
                }
              }
              Dout[m] = d;
            }
          }
          ++gc;
        }
#pragma unroll
        for (int m = 0; m < MT; ++m) Din[m] = Dout[m];
      }
      if constexpr (TRAIN)
        if (valid)
#pragma unroll
          for (int m = 0; m < MT; ++m) *reinterpret_cast<f32x4*>(erow<W>(a, 1, p) + 16 * m + 4 * g) = Din[m];
    }

    if constexpr (!TRAIN) {
      if constexpr (MODE != MODE_QUERY) {
        gx0 = sum_lane_groups(gx0);
        gx1 = sum_lane_groups(gx1);
        gx2 = sum_lane_groups(gx2);
      }
      store_outputs<MODE>(a, p, valid && g == 0, f, gx0, gx1, gx2, w0, w1, w2);
    }
  }
}

#define SDF_K32_INST(W, MODE) template __global__ void sdf_k32<W, MODE>(const KArgs);
#define SDF_K32_MODES(W) SDF_K32_INST(W, MODE_QUERY) SDF_K32_INST(W, MODE_GRAD) SDF_K32_INST(W, MODE_PROJECT) \
  SDF_K32_INST(W, MODE_TRAIN)
SDF_K32_MODES(64)
SDF_K32_MODES(128)
SDF_K32_MODES(256)

}  // namespace sdfc
