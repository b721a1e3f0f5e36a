// sdf_device.hpp -- gfx950 device helpers for the neural-SDF kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "sdf_layout.hpp"

namespace sdfc {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x8 __attribute__((ext_vector_type(8)));
typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));

enum { MODE_QUERY = 0, MODE_GRAD = 1, MODE_PROJECT = 2, MODE_TRAIN = 3 };
enum { PREC_FP32 = 0, PREC_BF16 = 1, PREC_FP16 = 2, PREC_BF16X3 = 3, PREC_FP8 = 4 };

// Everything a launch needs; passed by value in the kernel argument segment.
struct KArgs {
  const float* pts_in;   // [n][3]
  float* pts_out;        // [n][3] (collide_project: same as pts_in)
  int64_t n;
  float* sdf;            // [n] or null
  float* grad;           // [n][3] or null
  float* normal;         // [n][3] or null
  uint8_t* hit;          // [n] or null
  float eps;
  float bo;              // output bias
  const unsigned char* stream;  // packed fragments, forward then reverse
  const float* small;    // SmallLayout block
  float* scratch;        // FP32 kernels: per-slot sigma stack
  int L;                 // hidden layers
  int skip;              // 0 or 2..L
  int ff;                // 1: Fourier-feature input (layer 1 is an MFMA layer over gamma(x))
  // 16-bit kernels: the gradient copies of the layer-1 weights and of the skip
  // x-columns, and the reverse-sweep seed, as multiples of their forward copies
  float c_l1g, c_skg, c_wob;
  int nch;               // chunks streamed per tile
  int ntiles;            // ceil(n / 64)
  // fitting (MODE_TRAIN) only: per-point targets and the per-chunk workspace
  const float* target;   // [n] signed distances
  const float* bo_dev;   // output bias in device memory (the flat parameters)
  // FP8 operands: per-layer factors that undo the power-of-two operand scales
  // of the forward (fsc[l]) and reverse (rsc[l]) contraction of layer l
  float fsc[kLMax + 1];
  float rsc[kLMax + 1];
  // collider frame T = [A t; 0 1] (Sec. 4.2): the network is evaluated at
  // p' = A^{-1} (p - t) and its gradient returned as A^{-T} grad' (rigid = 0: identity)
  int rigid;
  float Ai[9];  // A^{-1}, row-major
  float tr[3];  // t
  float* ws_E;           // [L][n][W]: dLoss/dz_l per point
  float* ws_H;           // [L+1][n][W+16]: h_l, then x, y, z, 1, zeros (h_0 slot: x, y, z, 1 only)
  float* ws_U;           // [n][16]: dLoss/df, zeros
  float* ws_loss;        // [n]: |clamp(f) - clamp(s)| / n_total
  float delta;           // clamp of the L1 loss
  float inv_n;           // 1 / n_total (the whole batch, not the chunk)
  float inv_kappa;       // 1 / (beta log2 e): h = r / kappa
};

// Geometry of one network for the fitting kernels (flat parameter layout).
struct TrainNet {
  int W, L, skip;
  float kappa;
  int64_t offW[kLMax + 1], offb[kLMax + 1], offo;  // offsets into the flat array
  __host__ __device__ int K(int l) const { return (l == 1 ? 3 : W) + (l == skip ? 3 : 0); }
};

// Global-memory views of a pointer.  Loads and stores through them are
// global_load / global_store rather than flat ones.  The compiler infers the
// address space of pointers that arrive as kernel arguments, but not of
// pointers read from a table in memory (the grouped kernels); flat loads
// also count against the LDS wait counter, so every wait for an LDS read
// would wait for the weight loads in flight as well.
template <class T>
__device__ __forceinline__ const __attribute__((address_space(1))) T* gmem(const T* p) {
  return (const __attribute__((address_space(1))) T*)(p);
}
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gmem(T* p) {
  return (__attribute__((address_space(1))) T*)(p);
}
// gmem(p) where GV, else p itself (kernels whose pointers are kernel
// arguments keep the compiler's own addressing).
template <bool GV, class T>
__device__ __forceinline__ auto gview(T* p) {
  if constexpr (GV)
    return gmem(p);
  else
    return p;
}

__device__ __forceinline__ unsigned lds_u32(const void* p) {
  return (unsigned)(uintptr_t)(__attribute__((address_space(3))) const void*)p;
}

// One 16-byte-per-lane global->LDS copy; the wave's 64 lanes fill 1 KB at
// the wave-uniform LDS byte address `lds` (lane i -> lds + 16 i).  Issued as
// inline asm so the compiler's wait-count bookkeeping does not serialise the
// prefetch: waits for these copies are placed by hand (vm_wait_barrier).
__device__ __forceinline__ void dma16(const void* g, unsigned lds) {
  asm volatile("s_mov_b32 m0, %1\n\tglobal_load_lds_dwordx4 %0, off" ::"v"(g), "s"(lds)
               : "memory", "m0");
}

// Wait until at most N vector-memory operations of this wave are pending and
// all of its LDS operations are done, then barrier the workgroup.
template <int N>
__device__ __forceinline__ void vm_wait_barrier() {
  asm volatile("s_waitcnt vmcnt(%0) lgkmcnt(0)\n\ts_barrier" ::"I"(N) : "memory");
}

// Workgroup barrier that orders LDS traffic only: every wave's LDS reads and
// writes are complete before any wave passes.  Unlike __syncthreads() it does
// not wait for this wave's outstanding global loads (weight prefetches for the
// next layer stay in flight across the barrier).
__device__ __forceinline__ void lds_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// Copy chunk `c` of the weight stream into ring slot c % kNBuf.
template <class G>
__device__ __forceinline__ void issue_chunk(const unsigned char* stream, int c, unsigned ring,
                                            int wave, int lane) {
  const unsigned char* src = stream + (size_t)c * G::CHUNK + wave * 1024 + lane * 16;
  const unsigned dst = ring + (unsigned)((c % kNBuf) * G::CHUNK) + wave * 1024;
#pragma unroll
  for (int j = 0; j < G::LPC; ++j) dma16(src + j * 4096, dst + j * 4096);
}

// Make chunk gc resident and visible to the whole workgroup, and refill the
// slot freed by chunk gc-1 with chunk gc+kNBuf-1.  Chunks gc+1..gc+kNBuf-2
// stay in flight.
template <class G>
__device__ __forceinline__ void chunk_acquire(int gc, int nch, const unsigned char* stream,
                                              unsigned ring, int wave, int lane) {
  const int later = nch - 1 - gc;  // chunks issued after gc, capped below
  if (later >= kNBuf - 2)
    vm_wait_barrier<(kNBuf - 2) * G::LPC>();
  else if (later == 1)
    vm_wait_barrier<G::LPC>();
  else
    vm_wait_barrier<0>();
  if (gc + kNBuf - 1 < nch) issue_chunk<G>(stream, gc + kNBuf - 1, ring, wave, lane);
}

// log2(1 + 2^y), the rescaled softplus, with hardware exp2/log2:
// max(y, 0) + log2(1 + 2^-|y|), where max(y, 0) = (y + |y|) / 2 exactly.
__device__ __forceinline__ float softplus2(float y) {
  const float e = __builtin_amdgcn_exp2f(-__builtin_fabsf(y));
  return __builtin_fmaf(y + __builtin_fabsf(y), 0.5f, __builtin_amdgcn_logf(1.0f + e));
}

template <int PREC>
__device__ __forceinline__ unsigned pack2(float a, float b) {
  f32x2 v = {a, b};
  if constexpr (PREC == PREC_BF16)
    return __builtin_bit_cast(unsigned, __builtin_convertvector(v, bf16x2));
  else
    return __builtin_bit_cast(unsigned, __builtin_convertvector(v, f16x2));
}

template <int PREC>
__device__ __forceinline__ void unpack2(unsigned u, float& a, float& b) {
  if constexpr (PREC == PREC_BF16) {
    a = __builtin_bit_cast(float, u << 16);
    b = __builtin_bit_cast(float, u & 0xffff0000u);
  } else {
    const f16x2 h = __builtin_bit_cast(f16x2, u);
    a = (float)h.x;
    b = (float)h.y;
  }
}

template <int PREC>
__device__ __forceinline__ f32x4 mfma16(u32x4 a, u32x4 b, f32x4 c) {
  if constexpr (PREC == PREC_BF16)
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                   __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
  else
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a),
                                                  __builtin_bit_cast(f16x8, b), c, 0, 0, 0);
}

// v_mfma_f32_16x16x128_f8f6f4 with E4M3 operands on both sides (no block
// scales): 32 bytes of A and of B per lane, K = 128.
__device__ __forceinline__ f32x4 mfma_fp8(u32x8 a, u32x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(__builtin_bit_cast(i32x8, a),
                                                          __builtin_bit_cast(i32x8, b), c, 0, 0, 0, 0, 0, 0);
}

// Four floats as four E4M3 bytes (round to nearest even), saturated to +-448.
__device__ __forceinline__ unsigned pack4_fp8(f32x4 v) {
  f32x4 c;
#pragma unroll
  for (int i = 0; i < 4; ++i) c[i] = __builtin_fminf(__builtin_fmaxf(v[i], -448.0f), 448.0f);
  unsigned w = __builtin_amdgcn_cvt_pk_fp8_f32(c[0], c[1], 0u, false);
  return __builtin_amdgcn_cvt_pk_fp8_f32(c[2], c[3], w, true);
}

__device__ __forceinline__ float sum_lane_groups(float v) {
  v += __shfl_xor(v, 16, 64);
  v += __shfl_xor(v, 32, 64);
  return v;
}

// World point -> the network's frame.
__device__ __forceinline__ void to_local(const KArgs& a, float& x0, float& x1, float& x2) {
  if (!a.rigid) return;
  const float d0 = x0 - a.tr[0], d1 = x1 - a.tr[1], d2 = x2 - a.tr[2];
  x0 = __builtin_fmaf(a.Ai[0], d0, __builtin_fmaf(a.Ai[1], d1, a.Ai[2] * d2));
  x1 = __builtin_fmaf(a.Ai[3], d0, __builtin_fmaf(a.Ai[4], d1, a.Ai[5] * d2));
  x2 = __builtin_fmaf(a.Ai[6], d0, __builtin_fmaf(a.Ai[7], d1, a.Ai[8] * d2));
}

// Final per-point outputs, shared by every kernel family.  Only lanes of group
// 0 (lanes 0..15) store; the other groups hold the same reduced values.
// x0..x2: the vertex as loaded (world frame).  g0..g2: gradient in the
// network's frame.
template <int MODE, bool GV = false>
__device__ __forceinline__ void store_outputs(const KArgs& a, int64_t p, bool store, float f,
                                              float g0, float g1, float g2, float x0, float x1,
                                              float x2) {
  if (!store) return;
  if (a.rigid) {  // grad_p f(A^{-1}(p - t)) = A^{-T} grad'
    const float h0 = a.Ai[0] * g0 + a.Ai[3] * g1 + a.Ai[6] * g2;
    const float h1 = a.Ai[1] * g0 + a.Ai[4] * g1 + a.Ai[7] * g2;
    const float h2 = a.Ai[2] * g0 + a.Ai[5] * g1 + a.Ai[8] * g2;
    g0 = h0;
    g1 = h1;
    g2 = h2;
  }
  if constexpr (MODE == MODE_QUERY) {
    gview<GV>(a.sdf)[p] = f;
  } else if constexpr (MODE == MODE_GRAD) {
    if (a.sdf) gview<GV>(a.sdf)[p] = f;
    gview<GV>(a.grad)[3 * p] = g0;
    gview<GV>(a.grad)[3 * p + 1] = g1;
    gview<GV>(a.grad)[3 * p + 2] = g2;
  } else {
    const float nrm = __builtin_sqrtf(g0 * g0 + g1 * g1 + g2 * g2);
    float n0 = 0.0f, n1 = 0.0f, n2 = 0.0f;
    if (nrm > 0.0f) {
      const float inv = 1.0f / nrm;
      n0 = g0 * inv;
      n1 = g1 * inv;
      n2 = g2 * inv;
    }
    const bool hit = f < a.eps;  // NaN compares false
    if (hit && nrm > 0.0f) {
      const float t = a.eps - f;
      gview<GV>(a.pts_out)[3 * p] = x0 + t * n0;
      gview<GV>(a.pts_out)[3 * p + 1] = x1 + t * n1;
      gview<GV>(a.pts_out)[3 * p + 2] = x2 + t * n2;
    }
    if (a.sdf) gview<GV>(a.sdf)[p] = f;
    if (a.normal) {
      gview<GV>(a.normal)[3 * p] = n0;
      gview<GV>(a.normal)[3 * p + 1] = n1;
      gview<GV>(a.normal)[3 * p + 2] = n2;
    }
    if (a.hit) gview<GV>(a.hit)[p] = hit ? 1 : 0;
  }
}

}  // namespace sdfc
