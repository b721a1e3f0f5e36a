// sdf_layout.hpp -- packed weight layout shared by the host packer and the
// gfx950 kernels of the neural-SDF collision path.
//
// The network (Sec. 3.1, Eq. 1) is evaluated in a rescaled form that folds
// the softplus sharpness beta and the base change to exp2/log2 into constants:
// with kappa = beta * log2(e), y_l = kappa z_l and r_l = kappa h_l satisfy
//   y_1 = (kappa W_1) x + kappa b_1,
//   y_l = W_l r_{l-1} (+ kappa W_l^x x at the skip layer) + kappa b_l,
//   r_l = log2(1 + 2^{y_l}) = max(y_l, 0) + log2(1 + 2^{-|y_l|}),
//   f   = (w_o / kappa) . r_L + b_o,
// so the hidden weights W_l (l >= 2) are used unchanged.  The derivative
// dr/dy = 2^y / (1 + 2^y) = sigmoid(beta z) = 1 - 2^{-r}, which lets the
// reverse sweep (Sec. 3.2, back-propagation) recover every sigmoid from the
// stored r without keeping z.  Reverse sweep: d_L = w_o (.) s_L;
// d_{l-1} = (W_l^T d_l) (.) s_{l-1}; grad f = W_1^T d_1 + (W_skip^x)^T d_skip.
// The kappa factors cancel in that product, so the gradient uses plain W_1.
//
// The 16-bit kernels carry d_l scaled by 2^{S_l} (S_l a per-layer integer
// chosen at pack time) so FP16 operands neither overflow nor underflow; the
// scale ratios are folded into the packed W^T fragments (exact powers of
// two) and undone in the FP32 layer-1 and skip gradient weights.
#pragma once

#include <cstdint>

namespace sdfc {

constexpr int kLMax = 8;        // deepest network the register-resident sweep holds
constexpr int kBlock = 256;     // threads per workgroup: 4 wave64, 16 points each
constexpr int kPtsPerWave = 16;
constexpr int kPtsPerBlock = 64;
constexpr int kNBuf = 4;        // LDS ring of weight chunks
constexpr int kFrag = 1024;     // one MFMA A-operand fragment: 64 lanes x 16 B

// Small FP32 block (floats), copied to LDS once per workgroup.  Feature j of
// a width-W layer; "float4" entries are {c0, c1, c2, c3}.
struct SmallLayout {
  int W;
  __host__ __device__ constexpr int l1() const { return 0; }            // W float4: kappa W1[j][0..2], kappa b1[j]
  __host__ __device__ constexpr int l1g() const { return 4 * W; }       // W float4: 2^-S_1 W1[j][0..2], 0
  __host__ __device__ constexpr int skf() const { return 8 * W; }       // W float4: kappa W_s[j][x,y,z], 0
  __host__ __device__ constexpr int skg() const { return 12 * W; }      // W float4: 2^-S_s W_s[j][x,y,z], 0
  __host__ __device__ constexpr int wof() const { return 16 * W; }      // W: w_o[j] / kappa
  __host__ __device__ constexpr int wob() const { return 17 * W; }      // W: 2^{S_L} w_o[j]
  __host__ __device__ constexpr int bias(int l) const { return 18 * W + (l - 2) * W; }  // kappa b_l, l >= 2
  __host__ __device__ constexpr int floats() const { return (18 + kLMax - 1) * W; }
};

// Workgroup shape of the 16-bit kernels, shared by the packer (the weight
// stream is ordered by wave), the launcher and the kernel.  NS = 1: plain
// 16-bit operands; NS = 2: BF16 hi/lo pairs; f8: E4M3 operands (wider
// weight fragments).  Widths from 128 run 8 waves (2 per SIMD) on 64 points;
// pairs (32; 16 at width 512) and width 512 (32) take fewer points so that
// the reverse-sweep stack and the operands of a wave still fit its registers.
__host__ __device__ constexpr int k16_waves(int W) { return W >= 128 ? 8 : 4; }
// Tile variant 1 (plain 16-bit collide_project at widths 128-512, picked by
// the autotuner): half the points of variant 0 and twice its weight-prefetch
// depth.
__host__ __device__ constexpr int k16_cols(int W, int NS, bool f8 = false, int var = 0) {
  const int c = W == 512 ? (NS == 1 ? 2 : 1) : (NS == 1 ? 4 : 2);
  return var == 1 && c > 1 ? c / 2 : c;
}
__host__ __device__ constexpr int k16_points(int W, int NS, bool f8 = false, int var = 0) {
  return 16 * k16_cols(W, NS, f8, var);
}
__host__ __device__ constexpr bool k16_has_variant(int W, int prec_16bit_plain) {
  return W >= 128 && prec_16bit_plain;
}

// Fragment geometry of one hidden layer.
//  16-bit (v_mfma_f32_16x16x32_{bf16,f16}): M-tiles of 16 output rows, K-blocks
//  of 32 inputs.  Fragment (mt, kb), lane = 16 g + row, element e (0..7) holds
//  A[16 mt + row][32 kb + 16 (e / 4) + 4 g + (e % 4)], the K order in which the
//  previous layer's accumulators land in registers, so activations chain from
//  one layer to the next without any shuffle.
//  FP32 (v_mfma_f32_16x16x4_f32): fragment (mt, m), lane = 16 g + row, element
//  i (0..3) holds A[16 mt + row][16 m + 4 g + i], i.e. the four K-blocks whose
//  B operands are accumulator register i of M-tile m.
template <int W, bool F32>
struct Geo {
  static constexpr int MT = W / 16;
  static constexpr int KB = F32 ? W / 16 : W / 32;   // fragments per M-tile row
  static constexpr int LAYER_BYTES = MT * KB * kFrag;
  static constexpr int CHUNK = LAYER_BYTES < 32768 ? LAYER_BYTES : 32768;
  static constexpr int CPL = LAYER_BYTES / CHUNK;     // chunks per layer
  static constexpr int CH_MT = CHUNK / (KB * kFrag);  // M-tiles per chunk
  static constexpr int LPC = CHUNK / (kBlock * 16);   // 16-byte DMA loads per thread per chunk
  static_assert(CH_MT >= 2 && CH_MT % 2 == 0, "M-tiles are processed in pairs");
  static_assert(LPC >= 1 && (kNBuf - 2) * LPC <= 63, "vmcnt range");
};

}  // namespace sdfc
