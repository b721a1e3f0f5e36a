// sdf_k16.hip -- fused neural-SDF query / gradient / collision kernel with
// 16-bit (BF16 or FP16) MFMA operands and FP32 accumulation, for gfx950.
//
// One workgroup takes a tile of points (64 for widths up to 256: 4 column
// tiles of 16) through the whole network.  The hidden features of every layer
// are split across the waves (8 waves from width 128, i.e. 2 per SIMD; 4
// below): wave w owns features [w W/NWV, (w+1) W/NWV) for all points of the
// tile.  Per hidden layer l >= 2 each wave computes its rows of
// z_l = W_l r_{l-1} with v_mfma_f32_16x16x32_{bf16,f16}: A = its own weight
// fragments, loaded straight from L2 into registers (each weight byte enters
// the CU once per tile), B = the previous layer's activations of all
// features, read from an LDS exchange buffer that every wave fills with its
// own rows (Sec. 3.1, Eq. 1).  The reverse sweep of Sec. 3.2 runs the same way
// over W_l^T: a wave owns the input-feature rows it produced in the forward
// pass, so the sigmoids it needs come from its own registers (1 - 2^{-r}, r
// stored as 16-bit).  Layer 1 (K = 3), the skip x-columns, the output layer,
// the normal (Eq. 2) and the move to the contact point (Eq. 3) are FP32 VALU;
// per-point sums across waves go through LDS.  One workgroup barrier per
// layer publishes the exchange buffer; at width 256 a wave's own rows form a
// whole K-block of the next contraction, whose MFMAs are issued from
// registers before that barrier.
#include <type_traits>

#include "sdf_device.hpp"

namespace sdfc {

// NS = 1: plain 16-bit operands.  NS = 2: every operand is carried as a BF16
// pair hi + lo (lo = bf16(v - hi)) and each product is hi*hi + lo*hi + hi*lo,
// which keeps about 16 significant bits (compensated "BF16x3").
template <int W, int NS, bool F8 = false, int VAR = 0>
struct GeoB {
  static constexpr int NWV = k16_waves(W);    // waves per workgroup
  static constexpr int NCT = k16_cols(W, NS, F8, VAR);  // column tiles of 16 points
  static constexpr int PTS = 16 * NCT;         // points per workgroup
  static constexpr int FW = W / NWV;           // features per wave
  static constexpr int MTW = FW / 16;          // M-tiles per wave
  static constexpr int KM = F8 ? 128 : 32;      // K per MFMA
  static constexpr int KB = W / KM;            // K-blocks per layer
  static constexpr int FRAG = F8 ? 2 * kFrag : kFrag;  // bytes of one operand fragment
  // (pairs: 3, a four-slot ring, the weights three K-steps ahead)
  static constexpr int DMAX = (W == 512 ? (F8 ? 2 : 1) : (NS == 2 ? 3 : 1)) * (VAR == 1 ? 2 : 1);
  static constexpr int D = KB < DMAX ? KB : DMAX;  // weight prefetch depth in K-steps
  // ring of weight fragments: step j uses slot j % R while step j + R - 1 is
  // loaded into its own slot; R divides KB so the slots line up across layers
  static constexpr int R0 = (D + 1) >= 8 ? 8 : (D + 1) >= 4 ? 4 : (D + 1) >= 2 ? 2 : 1;  // power of two
  static constexpr int R = R0 <= KB ? R0 : KB;
  static_assert((R & (R - 1)) == 0, "ring size");
  // r_1..r_LS of the stack live in LDS (the reverse sweep reads them last);
  // the rest stay in registers.
  static constexpr int LS = W == 256 ? 2 : (W > 256 ? (F8 ? 3 : 1) : 0);
  static constexpr int STK_BYTES = (LS > 0 ? LS : 1) * NWV * MTW * NCT * NS * 64 * 8;
  static constexpr int WAVE_BYTES = KB * MTW * NS * FRAG;  // one wave's slice of a layer
  static constexpr int LAYER_BYTES = NWV * WAVE_BYTES;
  static constexpr int ACT_BYTES = KB * NCT * FRAG;        // one exchange buffer part
  static constexpr int NS_ = NS;
  // The biases of layers 1..8 sit in LDS with the rest of the small block,
  // except for FP8 at width 512, whose LDS holds three layers of the stack
  // instead: there each wave reads its biases from L2 once per layer.
  static constexpr bool SM_BIAS = !(W == 512 && F8);
  static constexpr int SM_FLOATS = (SM_BIAS ? 17 : 9) * W;
  // LDS of one workgroup (byte offsets, 16-byte aligned): the double-buffered
  // exchange buffers, the small FP32 block (17 W floats), the points, the
  // LDS part of the reverse-sweep stack, the per-wave partial sums.
  static constexpr int OFF_ACT = 0;
  static constexpr int OFF_SM = OFF_ACT + 2 * NS * ACT_BYTES;
  static constexpr int OFF_XS = OFF_SM + SM_FLOATS * 4;
  static constexpr int OFF_STK = OFF_XS + PTS * 16;
  static constexpr int OFF_RED = OFF_STK + STK_BYTES;
  static constexpr int LDS_BYTES = OFF_RED + NWV * PTS * 16;
  static_assert(MTW >= 1 && KB >= 1 && KB % R == 0, "shape");
};

template <int PREC>
__device__ __forceinline__ uint2 pack4(f32x4 v) {
  return uint2{pack2<PREC>(v[0], v[1]), pack2<PREC>(v[2], v[3])};
}

template <int PREC>
__device__ __forceinline__ f32x4 unpack4(uint2 u) {
  f32x4 r;
  float a, b;
  unpack2<PREC>(u.x, a, b);
  r[0] = a;
  r[1] = b;
  unpack2<PREC>(u.y, a, b);
  r[2] = a;
  r[3] = b;
  return r;
}

// Address of weight fragment part ps (0 hi, 1 lo) of (K-step kb, local M-tile mt).
template <class G, class AT, bool GV>
__device__ __forceinline__ auto wfrag(const unsigned char* layer, int wave, int kb, int mt, int ps, int lane) {
  return gview<GV>(reinterpret_cast<const AT*>(layer + (size_t)wave * G::WAVE_BYTES +
                                               (size_t)((kb * G::MTW + mt) * G::NS_ + ps) * G::FRAG +
                                               lane * (int)sizeof(AT)));
}

// v as a BF16 pair: hi = bf16(v), lo = bf16(v - hi).
__device__ __forceinline__ void split4(f32x4 v, uint2& hi, uint2& lo) {
  hi = pack4<PREC_BF16>(v);
  const f32x4 h = unpack4<PREC_BF16>(hi);
  lo = pack4<PREC_BF16>(v - h);
}

// The whole per-workgroup pass over tile `tile` (points [tile PTS, tile PTS +
// PTS) of a.pts_in) of network `a`.
// LDS geometry of a (width, operand type, tile variant) configuration.
template <int W, int PREC, int VAR>
using GeoP = GeoB<W, PREC == PREC_BF16X3 ? 2 : 1, PREC == PREC_FP8, VAR>;

// GV: read and write global memory through explicit global-address views
// (the grouped kernels, whose arguments come from a table in memory).
template <int W, int PREC, int MODE, int VAR, bool GV = false>
__device__ __forceinline__ void k16_tile(const KArgs& a, int tile, unsigned char* lds, int tid) {
  constexpr int NS = PREC == PREC_BF16X3 ? 2 : 1;
  // FP8: E4M3 exchange operands (forward activations stored as r / 4), weights
  // scaled per layer by a power of two undone by a.fsc / a.rsc; the stack of r
  // for the reverse sweep stays BF16.
  constexpr bool F8 = PREC == PREC_FP8;
  constexpr int OP = (PREC == PREC_BF16X3 || F8) ? PREC_BF16 : PREC;  // 16-bit operand / stack type
  using G = GeoB<W, NS, F8, VAR>;
  using AT = std::conditional_t<F8, u32x8, u32x4>;  // one lane's share of an operand fragment
  constexpr int NWV = G::NWV, NT = 64 * NWV;
  constexpr SmallLayout SL{W};
  constexpr int MTW = G::MTW, KB = G::KB, NCT = G::NCT, R = G::R, PTS = G::PTS;

  // LDS, carved from the caller's buffer of G::LDS_BYTES (16-byte aligned)
  auto& act = *reinterpret_cast<unsigned char (*)[2][NS][G::ACT_BYTES]>(lds + G::OFF_ACT);
  // The small FP32 block in the compact form this kernel reads: [l1: 4W |
  // skf: 4W | wof: W | bias of layers 1..8: 8W]; the gradient copies of l1 and
  // skf and the reverse seed are these times per-network scalars (a.c_l1g,
  // a.c_skg, a.c_wob).  Layer 1's bias slot holds the Fourier net's bias.
  constexpr int C_L1 = 0, C_SKF = 4 * W, C_WOF = 8 * W, C_FLOATS = G::SM_FLOATS;
  auto c_bias = [](int l) { return 9 * W + (l - 1) * W; };
  static_assert(C_FLOATS * 4 == G::OFF_XS - G::OFF_SM, "small block size");
  float* sm = reinterpret_cast<float*>(lds + G::OFF_SM);
  f32x4* xs = reinterpret_cast<f32x4*>(lds + G::OFF_XS);  // the workgroup's points
  uint2* stk_lds = reinterpret_cast<uint2*>(lds + G::OFF_STK);
  auto& red = *reinterpret_cast<f32x4 (*)[NWV][PTS]>(lds + G::OFF_RED);  // per wave: f, grad x partials

  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int g = lane >> 4, col = lane & 15;
  const int L = a.L, skip = a.skip;
  const int64_t base = (int64_t)tile * PTS;
  // first layer on MFMA: 2, or 1 with Fourier input (its K = 2m = W inputs are gamma(x))
  const int nf = a.ff ? 1 : 2;
  const unsigned char* fwd = a.stream;  // layers nf..L, LAYER_BYTES each
  const unsigned char* rev = a.stream + (size_t)(L - nf + 1) * G::LAYER_BYTES;  // layers L..nf

  // ---- points (to LDS), small weights ----
  if (tid < PTS) {
    const int64_t p = base + tid;
    f32x4 v = {0.0f, 0.0f, 0.0f, 0.0f};
    if (p < a.n) {
      const auto* src = gview<GV>(a.pts_in);
      float x0 = src[3 * p], x1 = src[3 * p + 1], x2 = src[3 * p + 2];
      to_local(a, x0, x1, x2);
      v[0] = x0;
      v[1] = x1;
      v[2] = x2;
    }
    xs[tid] = v;
  }
  {
    const auto* src = gview<GV>(reinterpret_cast<const f32x4*>(a.small));
    f32x4* dst = reinterpret_cast<f32x4*>(sm);
    for (int i = tid; i < W; i += NT) {  // l1, skf: one float4 per feature
      dst[C_L1 / 4 + i] = src[SL.l1() / 4 + i];
      dst[C_SKF / 4 + i] = src[SL.skf() / 4 + i];
    }
    for (int i = tid; i < W / 4; i += NT) {  // wof, layer-1 bias (Fourier), biases 2..8
      dst[C_WOF / 4 + i] = src[SL.wof() / 4 + i];
      if constexpr (G::SM_BIAS) dst[c_bias(1) / 4 + i] = src[SL.l1g() / 4 + i];
    }
    if constexpr (G::SM_BIAS)
      for (int i = tid; i < (kLMax - 1) * W / 4; i += NT) dst[c_bias(2) / 4 + i] = src[SL.bias(2) / 4 + i];
  }


  // feature index of (local M-tile mt, lane group g, element i)
  auto feat = [&](int mt, int i) { return 16 * (MTW * wave + mt) + 4 * g + i; };
  // LDS byte offset of this lane's half-fragment for global M-tile of local mt, tile ct
  auto act_off = [&](int mt, int ct) {
    const int m = MTW * wave + mt;
    return ((m >> 1) * NCT + ct) * kFrag + lane * 16 + 8 * (m & 1);
  };
  // FP8 exchange layout: the fragment of (K-block of 128, column tile) is
  // 8 / MTW planes of 64 lanes x 4 MTW bytes; plane p holds the operand bytes
  // of M-tiles 8 kb + p MTW .. 8 kb + p MTW + MTW - 1 (one wave's rows), so a
  // wave writes one contiguous 4 MTW-byte chunk per lane (free of bank
  // conflicts), and a lane's 32-byte B operand is its chunks of the 8 / MTW
  // planes in plane order.
  constexpr int PW = 4 * MTW;     // bytes per lane per plane
  constexpr int NPL = 32 / PW;    // planes per fragment
  auto f8_off = [&](int ct) {
    const int m0 = MTW * wave;
    return ((m0 >> 3) * NCT + ct) * G::FRAG + ((m0 & 7) / MTW) * 64 * PW + lane * PW;
  };
  unsigned f8w[F8 ? NCT : 1][F8 ? MTW : 1] = {};  // E4M3 words of the wave's M-tiles, per column tile
  // The wave's rows cover whole K-blocks of the next contraction when MTW is
  // even: K-block kb0 + j holds local M-tiles 2j, 2j + 1 (see act_off).
  constexpr int NOWN = (NS == 1 && !F8 && W != 512 && MTW % 2 == 0) ? MTW / 2 : 0;
  const int kb0 = wave * NOWN;
  u32x4 ownB[NOWN > 0 ? NOWN : 1][NCT][NS] = {};

  // first weight fragments (forward layer 2), in the wave's K-block order
  AT Aq[R][MTW][NS] = {};
#pragma unroll
  for (int s = 0; s < R - 1; ++s)
#pragma unroll
    for (int mt = 0; mt < MTW; ++mt)
#pragma unroll
      for (int ps = 0; ps < NS; ++ps) Aq[s][mt][ps] = *wfrag<G, AT, GV>(fwd, wave, (kb0 + s) & (KB - 1), mt, ps, lane);
  __syncthreads();

  // r_l of the wave's rows, l = LS+1..L-1, in registers: as the operand tuples
  // of the wave's own K-blocks (stq, NOWN > 0) or per M-tile (stk).
  u32x4 stq[kLMax][NOWN > 0 ? NOWN : 1][NCT][NS] = {};
  uint2 stk[kLMax][MTW][NCT][NS] = {};
  auto stk_at = [&](int l, int mt, int ct, int ps) -> uint2& {
    return stk_lds[(((((l - 1) * NWV + wave) * MTW + mt) * NCT + ct) * NS + ps) * 64 + lane];
  };
  auto keep_own = [&](int l) {  // after layer l's epilogue: stack the own tuples
    if constexpr (NOWN > 0)
      if (l > G::LS)
#pragma unroll
        for (int j = 0; j < NOWN; ++j)
#pragma unroll
          for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
            for (int ps = 0; ps < NS; ++ps) stq[l][j][ct][ps] = ownB[j][ct][ps];
  };
  auto stacked = [&](int l, int mt, int ct, int ps) -> uint2 {
    if (l <= G::LS) return stk_at(l, mt, ct, ps);
    if constexpr (NOWN > 0) {
      const u32x4 q = stq[l][mt / 2][ct][ps];
      return (mt & 1) ? uint2{q[2], q[3]} : uint2{q[0], q[1]};
    } else {
      return stk[l][mt][ct][ps];
    }
  };
  // Store v (FP32) as the wave's operand rows: 16-bit (NS = 1) or a BF16 pair.
  // keep_l: stack layer to record v in (0: none).
  auto put = [&](unsigned char* out, int mt, int ct, f32x4 v, int keep_l) {
    if constexpr (F8) {
      f8w[ct][mt] = pack4_fp8(keep_l > 0 ? v * 0.25f : v);
      if (mt == MTW - 1) {  // the wave's chunk of this column tile is complete
        unsigned char* dst = out + f8_off(ct);
        if constexpr (MTW == 1) {
          *reinterpret_cast<unsigned*>(dst) = f8w[ct][0];
        } else if constexpr (MTW == 2) {
          *reinterpret_cast<uint2*>(dst) = uint2{f8w[ct][0], f8w[ct][1]};
        } else {
          static_assert(MTW == 4, "FP8 chunk");
          *reinterpret_cast<u32x4*>(dst) = u32x4{f8w[ct][0], f8w[ct][1], f8w[ct][2], f8w[ct][3]};
        }
      }
      if (keep_l > 0) {
        const uint2 q = pack4<PREC_BF16>(v);
        if (keep_l <= G::LS)
          stk_at(keep_l, mt, ct, 0) = q;
        else
          stk[keep_l][mt][ct][0] = q;
      }
      return;
    }
    uint2 p[NS];
    if constexpr (NS == 1)
      p[0] = pack4<OP>(v);
    else
      split4(v, p[0], p[NS - 1]);
#pragma unroll
    for (int ps = 0; ps < NS; ++ps) {
      *reinterpret_cast<uint2*>(out + ps * G::ACT_BYTES + act_off(mt, ct)) = p[ps];
      if constexpr (NOWN > 0) {
        ownB[mt / 2][ct][ps][2 * (mt & 1)] = p[ps].x;
        ownB[mt / 2][ct][ps][2 * (mt & 1) + 1] = p[ps].y;
      }
      if (keep_l > 0 && keep_l <= G::LS)
        stk_at(keep_l, mt, ct, ps) = p[ps];
      else if (NOWN == 0 && keep_l > G::LS)
        stk[keep_l][mt][ct][ps] = p[ps];
    }
  };

  // Per-point partial sums of this wave (f and grad x) go to red[wave]: the lane
  // groups are summed with shuffles, then lanes 0..15 write or accumulate.
  auto flush = [&](int ct, f32x4 v, bool accumulate) {
#pragma unroll
    for (int c = 0; c < 4; ++c) v[c] = sum_lane_groups(v[c]);
    if (g == 0) {
      if (accumulate) v += red[wave][16 * ct + col];
      red[wave][16 * ct + col] = v;
    }
  };

  // b_j . x + phase_j of Fourier feature j, reduced to [-1/2, 1/2] revolutions
  auto ff_arg = [&](const f32x4& b, const f32x4& x) {
    const float v = __builtin_fmaf(b.x, x[0], __builtin_fmaf(b.y, x[1], __builtin_fmaf(b.z, x[2], b.w)));
    return v - __builtin_rintf(v);
  };
  if (!a.ff) {
    // ---- layer 1: y = kappa (W1 x + b1) ----
#pragma unroll
    for (int mt = 0; mt < MTW; ++mt) {
      f32x4 w4[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) w4[i] = *reinterpret_cast<const f32x4*>(&sm[C_L1 + 4 * feat(mt, i)]);
#pragma unroll
      for (int ct = 0; ct < NCT; ++ct) {
        const f32x4 x = xs[16 * ct + col];
        f32x4 r;
#pragma unroll
        for (int i = 0; i < 4; ++i)
          r[i] = softplus2(__builtin_fmaf(w4[i].x, x[0], __builtin_fmaf(w4[i].y, x[1], __builtin_fmaf(w4[i].z, x[2], w4[i].w))));
        put(&act[0][0][0], mt, ct, r, 1);
      }
    }
    keep_own(1);
  } else {
    // ---- Fourier input: gamma_j(x) = sin(2 pi (b_j . x + phase_j)), phase 1/4 for the cosines ----
#pragma unroll
    for (int mt = 0; mt < MTW; ++mt) {
      f32x4 b4[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) b4[i] = *reinterpret_cast<const f32x4*>(&sm[C_L1 + 4 * feat(mt, i)]);
#pragma unroll
      for (int ct = 0; ct < NCT; ++ct) {
        const f32x4 x = xs[16 * ct + col];
        f32x4 gm;
#pragma unroll
        for (int i = 0; i < 4; ++i) gm[i] = __builtin_amdgcn_sinf(ff_arg(b4[i], x));  // sin(2 pi v)
        put(&act[1][0][0], mt, ct, gm, 0);
      }
    }
  }

  // One hidden layer's contraction for this wave: acc[mt][ct] += A(mt, kb) B(kb, ct).
  // The K-blocks are taken in the order kb0, kb0 + 1, ... (mod KB).  When the
  // wave's own rows form whole K-blocks (OWN), those come first, straight from
  // the registers `put` filled, and are issued before the workgroup barrier
  // that publishes the other waves' rows, so they run while the barrier
  // resolves and the first LDS reads are in flight.  Each step first issues
  // the loads of later steps (weights R - 1 steps ahead, the next layer's from
  // `next` (nullptr: nothing follows); activations one step ahead), then its
  // MFMAs; a scheduling barrier keeps the loads ahead of the MFMAs.
  auto contract = [&](f32x4 (&acc)[MTW][NCT], const unsigned char* in, const unsigned char* layer,
                      const unsigned char* next) {
    auto kbi = [&](int j) { return (kb0 + j) & (KB - 1); };
    // raised wave priority while issuing MFMAs: when the other wave on the
    // SIMD is in its epilogue, the MFMA stream goes first (about 0.5 %)
    __builtin_amdgcn_s_setprio(1);
    // weights of step j + R - 1 into their ring slot
    auto prefetchA = [&](int j) {
      const int nk = j + R - 1;
      if (nk < KB) {
#pragma unroll
        for (int mt = 0; mt < MTW; ++mt)
#pragma unroll
          for (int ps = 0; ps < NS; ++ps) Aq[nk % R][mt][ps] = *wfrag<G, AT, GV>(layer, wave, kbi(nk), mt, ps, lane);
      } else if (next) {
#pragma unroll
        for (int mt = 0; mt < MTW; ++mt)
#pragma unroll
          for (int ps = 0; ps < NS; ++ps) Aq[nk % R][mt][ps] = *wfrag<G, AT, GV>(next, wave, kbi(nk - KB), mt, ps, lane);
      }
    };
    auto step = [&](int j, const AT (&B)[NCT][NS]) {
      const auto& Acur = Aq[j % R];
#pragma unroll
      for (int mt = 0; mt < MTW; ++mt)
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) {
          if constexpr (F8) {
            acc[mt][ct] = mfma_fp8(Acur[mt][0], B[ct][0], acc[mt][ct]);
          } else {
            if constexpr (NS == 2) {  // small cross terms first
              acc[mt][ct] = mfma16<OP>(Acur[mt][1], B[ct][0], acc[mt][ct]);
              acc[mt][ct] = mfma16<OP>(Acur[mt][0], B[ct][1], acc[mt][ct]);
            }
            acc[mt][ct] = mfma16<OP>(Acur[mt][0], B[ct][0], acc[mt][ct]);
          }
        }
    };
    if constexpr (NOWN > 0)
#pragma unroll
      for (int j = 0; j < NOWN; ++j) {
        prefetchA(j);
        step(j, ownB[j]);
      }
    lds_barrier();
    // B operands of K-steps j (in use) and j + 1 (in flight); single-operand
    // types at width 512 load each step's operands just before its MFMAs
    // instead, which keeps their 32-point tile within the registers (the
    // other wave on the SIMD covers the LDS latency)
    constexpr int NB = (W == 512 && NS == 1) ? 1 : 2;
    AT Bv[NB][NCT][NS];
    auto loadB = [&](AT (&dst)[NCT][NS], int j) {
#pragma unroll
      for (int ct = 0; ct < NCT; ++ct) {
        if constexpr (F8) {  // the lane's chunks of the NPL planes
          const unsigned char* src = in + (kbi(j) * NCT + ct) * G::FRAG + lane * PW;
#pragma unroll
          for (int pl = 0; pl < NPL; ++pl) {
            const unsigned char* c = src + pl * 64 * PW;
            if constexpr (MTW == 1) {
              dst[ct][0][pl] = *reinterpret_cast<const unsigned*>(c);
            } else if constexpr (MTW == 2) {
              const uint2 w = *reinterpret_cast<const uint2*>(c);
              dst[ct][0][2 * pl] = w.x;
              dst[ct][0][2 * pl + 1] = w.y;
            } else {
              const u32x4 w = *reinterpret_cast<const u32x4*>(c);
#pragma unroll
              for (int e = 0; e < 4; ++e) dst[ct][0][4 * pl + e] = w[e];
            }
          }
        } else {
#pragma unroll
          for (int ps = 0; ps < NS; ++ps)
            dst[ct][ps] = *reinterpret_cast<const AT*>(in + ps * G::ACT_BYTES + (kbi(j) * NCT + ct) * G::FRAG +
                                                       lane * (int)sizeof(AT));
        }
      }
    };
    if constexpr (NB == 2) loadB(Bv[0], NOWN);
#pragma unroll
    for (int j = NOWN; j < KB; ++j) {
      prefetchA(j);
      if constexpr (NB == 2) {
        if (j + 1 < KB) loadB(Bv[(j + 1 - NOWN) & 1], j + 1);
      } else {
        loadB(Bv[0], j);
      }
      __builtin_amdgcn_sched_barrier(0);
      step(j, Bv[(j - NOWN) & (NB - 1)]);
    }
    __builtin_amdgcn_s_setprio(0);
  };

  // ---- hidden layers nf..L, forward ----
#pragma unroll
  for (int l = 1; l <= kLMax; ++l) {
    if (l > L) break;
    if (l < nf) continue;
    const int t = l - 1;  // exchange step: read act[(t-1)&1], write act[t&1]
    const unsigned char* in = &act[(t - 1) & 1][0][0];
    unsigned char* out = &act[t & 1][0][0];
    const unsigned char* layer = fwd + (size_t)(l - nf) * G::LAYER_BYTES;
    const unsigned char* next =
        (l < L) ? layer + G::LAYER_BYTES : (MODE != MODE_QUERY ? rev : nullptr);
    f32x4 acc[MTW][NCT];
#pragma unroll
    for (int mt = 0; mt < MTW; ++mt) {
      const int fo = 16 * (MTW * wave + mt) + 4 * g;
      f32x4 b;
      if constexpr (G::SM_BIAS)
        b = *reinterpret_cast<const f32x4*>(&sm[c_bias(l) + fo]);
      else
        b = *gview<GV>(reinterpret_cast<const f32x4*>(a.small + (l == 1 ? SL.l1g() : SL.bias(l)) + fo));
#pragma unroll
      for (int ct = 0; ct < NCT; ++ct) acc[mt][ct] = b;
    }
    if (l == skip) {
#pragma unroll
      for (int mt = 0; mt < MTW; ++mt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const f32x4 w = *reinterpret_cast<const f32x4*>(&sm[C_SKF + 4 * feat(mt, i)]);
#pragma unroll
          for (int ct = 0; ct < NCT; ++ct) {
            const f32x4 x = xs[16 * ct + col];
            acc[mt][ct][i] = __builtin_fmaf(w.x, x[0], __builtin_fmaf(w.y, x[1], __builtin_fmaf(w.z, x[2], acc[mt][ct][i])));
          }
        }
    }
    contract(acc, in, layer, next);
    if (l < L) {
#pragma unroll
      for (int mt = 0; mt < MTW; ++mt)
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) {
          f32x4 r;
#pragma unroll
          for (int i = 0; i < 4; ++i) r[i] = softplus2(F8 ? acc[mt][ct][i] * a.fsc[l] : acc[mt][ct][i]);
          put(out, mt, ct, r, l);
        }
      keep_own(l);
    } else {
      // output layer f = (w_o/kappa) . r_L and the reverse-sweep seed
      // d_L = w_o (1 - 2^-r_L); SKIPG: layer L is also the skip layer.
      auto last_epi = [&](auto SKIPG) {
        f32x4 part[NCT];  // f, grad x partials of this wave's features
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) part[ct] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int mt = 0; mt < MTW; ++mt) {
          const f32x4 wf = *reinterpret_cast<const f32x4*>(&sm[C_WOF + 16 * (MTW * wave + mt) + 4 * g]);
          const f32x4 wb = wf * a.c_wob;
          f32x4 wg[4];
          if constexpr (decltype(SKIPG)::value)
#pragma unroll
            for (int i = 0; i < 4; ++i) wg[i] = *reinterpret_cast<const f32x4*>(&sm[C_SKF + 4 * feat(mt, i)]) * a.c_skg;
#pragma unroll
          for (int ct = 0; ct < NCT; ++ct) {
            f32x4 d;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const float r = softplus2(F8 ? acc[mt][ct][i] * a.fsc[l] : acc[mt][ct][i]);
              part[ct][0] = __builtin_fmaf(wf[i], r, part[ct][0]);
              d[i] = __builtin_fmaf(-wb[i], __builtin_amdgcn_exp2f(-r), wb[i]);
            }
            if constexpr (MODE != MODE_QUERY) {
              if constexpr (decltype(SKIPG)::value) {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                  part[ct][1] = __builtin_fmaf(wg[i].x, d[i], part[ct][1]);
                  part[ct][2] = __builtin_fmaf(wg[i].y, d[i], part[ct][2]);
                  part[ct][3] = __builtin_fmaf(wg[i].z, d[i], part[ct][3]);
                }
              }
              put(out, mt, ct, d, 0);
            }
          }
        }
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) flush(ct, part[ct], false);
      };
      if (MODE != MODE_QUERY && l == skip)
        last_epi(std::true_type{});
      else
        last_epi(std::false_type{});
    }
  }

  // ---- reverse sweep over W_l^T, l = L..nf ----
  if constexpr (MODE != MODE_QUERY) {
#pragma unroll
    for (int l = kLMax; l >= 1; --l) {
      if (l > L || l < nf) continue;
      const int t = 2 * L - l;
      const unsigned char* in = &act[(t - 1) & 1][0][0];
      unsigned char* out = &act[t & 1][0][0];
      const unsigned char* layer = rev + (size_t)(L - l) * G::LAYER_BYTES;
      const unsigned char* next = (l > nf) ? layer + G::LAYER_BYTES : nullptr;
      f32x4 acc[MTW][NCT];
#pragma unroll
      for (int mt = 0; mt < MTW; ++mt)
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) acc[mt][ct] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
      contract(acc, in, layer, next);
      // d_{l-1} = g (1 - 2^-r_{l-1}); TOX: fold d_{l-1} into grad x through the
      // layer-1 weights (l == 2) or the skip layer's x-columns (l - 1 == skip).
      auto bwd_epi = [&](auto TOX) {
        f32x4 part[NCT];  // grad x partials (components 1..3)
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) part[ct] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int mt = 0; mt < MTW; ++mt) {
          f32x4 wg[4];
          if constexpr (decltype(TOX)::value) {
            const int off = (l == 2) ? C_L1 : C_SKF;
            const float c = (l == 2) ? a.c_l1g : a.c_skg;
#pragma unroll
            for (int i = 0; i < 4; ++i) wg[i] = *reinterpret_cast<const f32x4*>(&sm[off + 4 * feat(mt, i)]) * c;
          }
#pragma unroll
          for (int ct = 0; ct < NCT; ++ct) {
            uint2 q[NS];
#pragma unroll
            for (int ps = 0; ps < NS; ++ps) q[ps] = stacked(l - 1, mt, ct, ps);
            f32x4 r = unpack4<OP>(q[0]);
            if constexpr (NS == 2) r += unpack4<OP>(q[1]);
            f32x4 d;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const float gi = F8 ? acc[mt][ct][i] * a.rsc[l] : acc[mt][ct][i];
              d[i] = __builtin_fmaf(-gi, __builtin_amdgcn_exp2f(-r[i]), gi);
            }
            if constexpr (decltype(TOX)::value) {
#pragma unroll
              for (int i = 0; i < 4; ++i) {
                part[ct][1] = __builtin_fmaf(wg[i].x, d[i], part[ct][1]);
                part[ct][2] = __builtin_fmaf(wg[i].y, d[i], part[ct][2]);
                part[ct][3] = __builtin_fmaf(wg[i].z, d[i], part[ct][3]);
              }
            }
            if (l > 2 || a.ff) put(out, mt, ct, d, 0);
          }
        }
        if constexpr (decltype(TOX)::value)
#pragma unroll
          for (int ct = 0; ct < NCT; ++ct) flush(ct, part[ct], true);
      };
      // l == 1 (Fourier input): acc = d f / d gamma for this wave's features;
      // grad x += sum_j acc_j 2 pi cos(2 pi (b_j . x + phase_j)) b_j
      auto ff_epi = [&]() {
        f32x4 part[NCT];
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) part[ct] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int mt = 0; mt < MTW; ++mt) {
          f32x4 b4[4];
#pragma unroll
          for (int i = 0; i < 4; ++i) b4[i] = *reinterpret_cast<const f32x4*>(&sm[C_L1 + 4 * feat(mt, i)]);
#pragma unroll
          for (int ct = 0; ct < NCT; ++ct) {
            const f32x4 x = xs[16 * ct + col];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const float s = acc[mt][ct][i] * 6.28318530717958647f * __builtin_amdgcn_cosf(ff_arg(b4[i], x));
              part[ct][1] = __builtin_fmaf(b4[i].x, s, part[ct][1]);
              part[ct][2] = __builtin_fmaf(b4[i].y, s, part[ct][2]);
              part[ct][3] = __builtin_fmaf(b4[i].z, s, part[ct][3]);
            }
          }
        }
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) flush(ct, part[ct], true);
      };
      if (l == 1)
        ff_epi();
      else if ((l == 2 && !a.ff) || l - 1 == skip)
        bwd_epi(std::true_type{});
      else
        bwd_epi(std::false_type{});
    }
  }

  // ---- per-point sums across waves; waves 0..NCT-1 finish column tile `wave` ----
  lds_barrier();
  if (wave < NCT) {
    f32x4 s = red[0][16 * wave + col];
#pragma unroll
    for (int w = 1; w < NWV; ++w) s += red[w][16 * wave + col];
    f32x4 x = xs[16 * wave + col];
    const int64_t p = base + 16 * wave + col;
    if constexpr (F8) {
      // E4M3 conversion saturates, so a NaN vertex would come out with a
      // finite f: give it what the other operand types give, f = NaN and a
      // zero gradient (never a hit, not moved)
      if (x[0] != x[0] || x[1] != x[1] || x[2] != x[2]) s = f32x4{__builtin_nanf(""), 0.0f, 0.0f, 0.0f};
    }
    if (a.rigid && p < a.n) {  // the vertex moves in the world frame
      const auto* src = gview<GV>(a.pts_in);
      x[0] = src[3 * p];
      x[1] = src[3 * p + 1];
      x[2] = src[3 * p + 2];
    }
    store_outputs<MODE, GV>(a, p, p < a.n && g == 0, s[0] + a.bo, s[1], s[2], s[3], x[0], x[1], x[2]);
  }
}

#define K16_WG_SIZE(W) \
  __attribute__((amdgpu_flat_work_group_size(64 * k16_waves(W), 64 * k16_waves(W)), amdgpu_waves_per_eu(2)))

template <int W, int PREC, int MODE, int VAR>
__global__ void K16_WG_SIZE(W) sdf_k16(const KArgs a) {
  __shared__ __attribute__((aligned(16))) unsigned char lds[GeoP<W, PREC, VAR>::LDS_BYTES];
  k16_tile<W, PREC, MODE, VAR>(a, blockIdx.x, lds, threadIdx.x);
}

// Several networks of one width in one launch: workgroup b runs tile
// b - tile_start[i] of network i, where tile_start[i] <= b < tile_start[i+1].
template <int W, int PREC, int MODE, int VAR>
__global__ void K16_WG_SIZE(W) sdf_k16_group(const KArgs* __restrict__ nets,
                                             const int* __restrict__ tile_start, int n_nets,
                                             int tile0) {
  const int b = tile0 + (int)blockIdx.x;
  int lo = 0, hi = n_nets - 1;  // last i with tile_start[i] <= b
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (tile_start[mid] <= b) lo = mid; else hi = mid - 1;
  }
  const int i = __builtin_amdgcn_readfirstlane(lo);
  __shared__ __attribute__((aligned(16))) unsigned char lds[GeoP<W, PREC, VAR>::LDS_BYTES];
  const KArgs a = nets[i];  // a private copy: loaded once, not again after every barrier
  k16_tile<W, PREC, MODE, VAR, true>(a, b - tile_start[i], lds, threadIdx.x);
}

// Several networks of widths 128-512 (512-thread workgroups) in one
// persistent launch: every workgroup takes work items -- one tile of one
// network -- from the counter ctr[0] until none are left.  Network i owns
// items item_start[i] .. item_start[i + 1] - 1 (its tiles in order); items
// run network by network, so the workgroups in flight mostly share one
// network's weights in L2.  The item table and the widths sit in LDS, the
// current network's arguments too (copied when the network changes), and
// each workgroup fetches its next item number while it works on the current
// one, so nothing but LDS stands between two tiles.  The last workgroup to
// run out of items sets both counters back to 0 for the next pass (ctr[1]
// counts the workgroups that are done), so a pass needs no separate reset and
// can be captured into a graph.
constexpr int kPersistMaxNets = 512;
template <int PREC>
__global__ void K16_WG_SIZE(256) sdf_k16_persist(const KArgs* __restrict__ nets, const int* __restrict__ width,
                                                 const int* __restrict__ item_start, int n_nets,
                                                 int* __restrict__ ctr) {
  constexpr int B128 = GeoP<128, PREC, 0>::LDS_BYTES, B256 = GeoP<256, PREC, 0>::LDS_BYTES,
                B512 = GeoP<512, PREC, 0>::LDS_BYTES;
  constexpr int BMAX = B128 > B256 ? (B128 > B512 ? B128 : B512) : (B256 > B512 ? B256 : B512);
  __shared__ __attribute__((aligned(16))) unsigned char lds[BMAX];
  __shared__ int tab[2 * kPersistMaxNets + 1];  // item_start[0..n_nets], then width[0..n_nets-1]
  __shared__ int next_s;  // the next item number
  for (int t = threadIdx.x; t <= n_nets; t += blockDim.x) {
    tab[t] = item_start[t];
    if (t < n_nets) tab[n_nets + 1 + t] = width[t];
  }
  if (threadIdx.x == 0) next_s = atomicAdd(&ctr[0], 1);
  __syncthreads();
  const int n_items = tab[n_nets];
  for (;;) {
    const int item = next_s;
    if (item >= n_items) break;
    int nxt = 0;
    if (threadIdx.x == 0) nxt = atomicAdd(&ctr[0], 1);  // used after this item
    int lo = 0, hi = n_nets - 1;  // last i with item_start[i] <= item
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (tab[mid] <= item) lo = mid; else hi = mid - 1;
    }
    const int i = __builtin_amdgcn_readfirstlane(lo);
    const KArgs& ka = nets[i];  // uniform address: read through the scalar cache
    const int tile = item - tab[i];
    // The thread index passes through an opaque move every item, so nothing
    // derived from it is hoisted out of this loop: kept live across all three
    // tile bodies, those values would not fit the registers.
    int tid;
    asm volatile("v_mov_b32 %0, %1" : "=v"(tid) : "v"((int)threadIdx.x));
    switch (__builtin_amdgcn_readfirstlane(tab[n_nets + 1 + i])) {
      case 128: k16_tile<128, PREC, MODE_PROJECT, 0, true>(ka, tile, lds, tid); break;
      case 256: k16_tile<256, PREC, MODE_PROJECT, 0, true>(ka, tile, lds, tid); break;
      default: k16_tile<512, PREC, MODE_PROJECT, 0, true>(ka, tile, lds, tid); break;
    }
    if (threadIdx.x == 0) next_s = nxt;
    __syncthreads();  // the next item is published; LDS is free for it
  }
  if (threadIdx.x == 0) {
    __threadfence();  // this workgroup's last fetch from ctr[0] comes first
    if (atomicAdd(&ctr[1], 1) == (int)gridDim.x - 1) {
      atomicExch(&ctr[0], 0);
      atomicExch(&ctr[1], 0);
    }
  }
}

#define SDF_K16_INST_V(W, PREC, MODE, VAR) \
  template __global__ void sdf_k16<W, PREC, MODE, VAR>(const KArgs); \
  template __global__ void sdf_k16_group<W, PREC, MODE, VAR>(const KArgs*, const int*, int, int);
#define SDF_K16_INST(W, PREC, MODE) SDF_K16_INST_V(W, PREC, MODE, 0)
#define SDF_K16_MODES(W, PREC) \
  SDF_K16_INST(W, PREC, MODE_QUERY) SDF_K16_INST(W, PREC, MODE_GRAD) SDF_K16_INST(W, PREC, MODE_PROJECT)

#if defined(SDF_K16_PERSIST)
template __global__ void sdf_k16_persist<SDF_K16_PREC>(const KArgs*, const int*, const int*, int, int*);
#endif

// The instantiations are split by hidden width and operand type so the build
// can compile this file once per pair in parallel (-DSDF_K16_WIDTH=64..512,
// -DSDF_K16_PREC=1..4, the PREC_* values); a macro left undefined selects every value.
#if defined(SDF_K16_WIDTH)
#define K16_W(W) (SDF_K16_WIDTH == (W))
#else
#define K16_W(W) 1
#endif
#if defined(SDF_K16_PREC)
#define K16_P(P) (SDF_K16_PREC == (P))
#else
#define K16_P(P) 1
#endif
#define K16_SEL(W, P) (K16_W(W) && K16_P(P))

#if K16_SEL(64, 1)
SDF_K16_MODES(64, PREC_BF16)
#endif
#if K16_SEL(64, 2)
SDF_K16_MODES(64, PREC_FP16)
#endif
#if K16_SEL(64, 3)
SDF_K16_MODES(64, PREC_BF16X3)
#endif
// widths 128..512 add FP8 operands and tile variant 1 of the plain 16-bit
// collision kernels (for the autotuner)
#if K16_SEL(128, 1)
SDF_K16_MODES(128, PREC_BF16)
SDF_K16_INST_V(128, PREC_BF16, MODE_PROJECT, 1)
#endif
#if K16_SEL(128, 2)
SDF_K16_MODES(128, PREC_FP16)
SDF_K16_INST_V(128, PREC_FP16, MODE_PROJECT, 1)
#endif
#if K16_SEL(128, 3)
SDF_K16_MODES(128, PREC_BF16X3)
#endif
#if K16_SEL(128, 4)
SDF_K16_MODES(128, PREC_FP8)
#endif
#if K16_SEL(256, 1)
SDF_K16_MODES(256, PREC_BF16)
SDF_K16_INST_V(256, PREC_BF16, MODE_PROJECT, 1)
#endif
#if K16_SEL(256, 2)
SDF_K16_MODES(256, PREC_FP16)
SDF_K16_INST_V(256, PREC_FP16, MODE_PROJECT, 1)
#endif
#if K16_SEL(256, 3)
SDF_K16_MODES(256, PREC_BF16X3)
#endif
#if K16_SEL(256, 4)
SDF_K16_MODES(256, PREC_FP8)
#endif
#if K16_SEL(512, 1)
SDF_K16_MODES(512, PREC_BF16)
SDF_K16_INST_V(512, PREC_BF16, MODE_PROJECT, 1)
#endif
#if K16_SEL(512, 2)
SDF_K16_MODES(512, PREC_FP16)
SDF_K16_INST_V(512, PREC_FP16, MODE_PROJECT, 1)
#endif
#if K16_SEL(512, 3)
SDF_K16_MODES(512, PREC_BF16X3)
#endif
#if K16_SEL(512, 4)
SDF_K16_MODES(512, PREC_FP8)
#endif

}  // namespace sdfc
