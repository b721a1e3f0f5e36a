/*
 * sdfcollide.h -- C ABI of the MI355X (gfx950) neural-SDF collision library.
 *
 * Method: Bertiche, Madadi, Escalera, "Neural Implicit Surfaces for Efficient
 * and Accurate Collisions in Physically Based Simulations" (arXiv 2110.01614).
 * A learned signed-distance MLP f: R^3 -> R (Sec. 3.1, Eq. 1) is evaluated at
 * every cloth vertex together with its analytic input gradient obtained by
 * back-propagation (Sec. 3.2); the normal is N = grad f / |grad f| (Eq. 2), a
 * vertex collides when f(p) < eps (Sec. 3.2), and a colliding vertex is moved
 * along N by (eps - f(p)), the contact-point offset of Eq. 3.  Interior is
 * negative, so the gradient points outward (Sec. 3.2).
 *
 * Conventions shared by every entry point:
 *  - Array arguments are DEVICE pointers (hipMalloc'd or torch CUDA tensors),
 *    caller-owned, contiguous, 4-byte aligned.  Points are float32 [n][3]
 *    array-of-structures.  The library never frees or retains them.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Work
 *    is enqueued asynchronously; device faults surface at the caller's sync.
 *  - Return value: SDF_OK (0) or a negative SDF_E* code.  Argument checks run
 *    on the host before anything is launched; on failure nothing is launched
 *    and sdf_last_error() (thread-local) describes the problem.
 *  - n == 0 returns SDF_OK and launches nothing; the array pointers may then
 *    be NULL.
 *  - Numerical policy: outputs are float32 whatever the internal precision; a
 *    NaN f is not a hit; |grad f| == 0 gives N = 0 and the vertex is not
 *    moved; a vertex that is not moved keeps its exact bit pattern.
 *  - The handle is immutable after creation: concurrent calls with one handle
 *    on different streams are allowed; sdf_net_destroy needs the caller to
 *    have synchronised every stream that used the handle.  SDF_FP32 handles
 *    keep one reverse-sweep scratch area, so their calls are ordered on the
 *    device instead of overlapping: a call issued on another stream than the
 *    previous call on the handle first waits (hipStreamWaitEvent) for that
 *    call.  While a stream is being captured into a graph, FP32 calls on one
 *    handle must all be issued on that stream.
 */
#ifndef SDFCOLLIDE_H
#define SDFCOLLIDE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  SDF_OK = 0,
  SDF_EINVAL = -1,       /* bad argument (null pointer, n < 0, non-finite eps, ...) */
  SDF_EUNSUPPORTED = -2, /* a network shape or precision the library has no kernel for */
  SDF_ENOMEM = -3,       /* device allocation failed in sdf_net_create */
  SDF_EDEVICE = -4       /* a HIP runtime call or launch failed */
};

/* Operand precision of the hidden-layer contractions (MFMA, FP32 accumulate).
 * SDF_BF16X3 carries every operand (weights, activations, back-propagated
 * errors) as a BF16 pair hi + lo and forms each product as hi*hi + lo*hi +
 * hi*lo: three BF16 MFMAs per product, about 16 significant bits.
 * SDF_FP8 uses OCP E4M3 operands (3 mantissa bits) on the K = 128 FP8 MFMA:
 * every layer's weights carry a power-of-two scale chosen at sdf_net_create
 * from the largest weight (largest scaled weight in (224, 448]), activations
 * enter as softplus output * beta * log2(e) / 4 and back-propagated errors
 * with the per-layer scales of the 16-bit paths, all saturated at +-448; the
 * stored activations of the reverse sweep stay BF16.  Widths 128-512.
 * Layer 1 (K = 3), the skip x-columns, the output layer, the normalisation
 * and the projection always run in FP32. */
enum { SDF_FP32 = 0, SDF_BF16 = 1, SDF_FP16 = 2, SDF_BF16X3 = 3, SDF_FP8 = 4 };

#define SDF_MAX_HIDDEN 16

/* Network shape (Sec. 3.1: one MLP per rigid object).  in_dim is 3, out_dim 1.
 * Hidden layer l (1-based) has width[l-1] units and softplus activation
 * softplus_beta(z) = log(1 + exp(beta z)) / beta.  If skip_layer = s > 0,
 * hidden layer s takes [h_{s-1}; x] (hidden features first, then x, y, z).
 * Fourier features: with fourier = m > 0 the network's input is
 * gamma(x) = [sin(2 pi B x), cos(2 pi B x)] (B an m x 3 matrix, fixed), layer 1
 * has K = 2m inputs and there is no skip input (skip_layer must be 0); this
 * build requires 2m == width and BF16, FP16 or BF16X3 operands.
 * The library has kernels for equal hidden widths of 64, 128, 256 or 512 (512:
 * 16-bit and FP8 precisions only; FP8: 128 and up), depth 2..8, skip 0 or
 * 2..depth; other shapes return SDF_EUNSUPPORTED. */
typedef struct {
  int32_t n_hidden;
  int32_t width[SDF_MAX_HIDDEN];
  int32_t skip_layer;
  float beta;
  int32_t precision;
  int32_t fourier; /* m > 0: Fourier-feature input (Sec. 3.1, Sec. 4.3), see below */
} sdf_net_desc;

typedef struct sdf_net sdf_net; /* opaque; owns device copies of packed weights */

/* Number of float32 parameters of `desc` in the flat layout below, or -1 if
 * the description is malformed.  Flat layout (the concatenation of every
 * nn.Linear weight then bias): for a Fourier net first B row-major [m][3];
 * then for l = 1..L, W_l row-major [width_l][K_l] then b_l[width_l], K_1 = 3
 * (2m with Fourier input), K_l = width_{l-1} (+3 at the skip layer); then
 * w_o[width_L], b_o. */
int64_t sdf_param_count(const sdf_net_desc* desc);

/* Packs `params_host` (HOST float32, n_params values, copied) for `device`
 * and returns a handle in *out.  Allocates all device memory the queries will
 * ever need (no allocation happens on the query path).  Errors: SDF_EINVAL
 * (null pointer, bad shape, n_params mismatch, non-finite beta or params),
 * SDF_EUNSUPPORTED, SDF_ENOMEM, SDF_EDEVICE. */
int sdf_net_create(const sdf_net_desc* desc, const float* params_host, size_t n_params,
                   int device, sdf_net** out);

/* Frees the handle and its device memory.  NULL is ignored. */
int sdf_net_destroy(sdf_net* net);

/* f(p) for n points (Sec. 3.1, Eq. 1).  pts: device float32 [n][3] (read);
 * sdf: device float32 [n] (written).  pts and sdf must not overlap. */
int sdf_query(const sdf_net* net, const float* pts, int64_t n, float* sdf, void* stream);

/* f(p) and the unnormalised input gradient grad f(p) by reverse-mode
 * back-propagation (Sec. 3.2).  sdf: device float32 [n] or NULL; grad: device
 * float32 [n][3] (required).  Outputs must not overlap pts. */
int sdf_query_grad(const sdf_net* net, const float* pts, int64_t n, float* sdf, float* grad,
                   void* stream);

/* The collision step of Sec. 3.2 for every vertex, in place: detect f < eps
 * (strict), N = grad f/|grad f| (Eq. 2), move hits to p + (eps - f) N (Eq. 3).
 * pts: device float32 [n][3] (read and overwritten).  sdf (f before the move,
 * [n]), normal ([n][3]) and hit (uint8 [n], 1 = f < eps) are optional device
 * outputs (NULL to skip) that must not overlap pts.  eps must be finite. */
int collide_project(const sdf_net* net, float* pts, int64_t n, float eps, float* sdf,
                    float* normal, uint8_t* hit, void* stream);

/* ---- a collider in its own frame (Sec. 4.2: moving a neural implicit surface) ----
 *
 * T: HOST pointer to a 4x4 row-major matrix [A t; 0 0 0 1] placing the network's
 * frame in the world (rotation and translation; any invertible A is accepted).
 * The network is evaluated at p' = A^{-1} (p - t); the gradient returned and
 * used for the normal is the gradient of p -> f(A^{-1}(p - t)), i.e.
 * A^{-T} grad f(p'), which for a rotation A is A grad f(p') as in Sec. 4.2; the
 * vertex moves in the world frame, p + (eps - f(p')) N.  The matrix is read
 * during the call (no retention).  Errors as the calls above, plus SDF_EINVAL
 * for a NULL, non-finite or singular T or a last row other than (0, 0, 0, 1).
 * Distances are only preserved by rigid T; a scaled A gives f(A^{-1}(p - t)). */
int sdf_query_rigid(const sdf_net* net, const float* T, const float* pts, int64_t n, float* sdf,
                    void* stream);
int sdf_query_grad_rigid(const sdf_net* net, const float* T, const float* pts, int64_t n, float* sdf,
                         float* grad, void* stream);
int collide_project_rigid(const sdf_net* net, const float* T, float* pts, int64_t n, float eps,
                          float* sdf, float* normal, uint8_t* hit, void* stream);

/* ---- several colliders per call (one network per rigid object, Sec. 3.1) ---- */

typedef struct sdf_group sdf_group; /* opaque; device tables of a fixed set of calls */

/* Binds n_nets networks (same device, same 16-bit or FP8 precision; widths may
 * differ) to their vertex buffers pts[i] (device float32 [counts[i]][3]) and
 * the contact offset eps, for repeated in-place collide_project passes over
 * all of them.  Buffers and counts are fixed for the life of the group, so a
 * pass can be captured into a HIP graph and replayed.  Allocates its device
 * tables here.  Errors: SDF_EINVAL, SDF_EUNSUPPORTED (FP32 networks),
 * SDF_ENOMEM, SDF_EDEVICE. */
int sdf_group_create(const sdf_net* const* nets, int n_nets, float* const* pts,
                     const int64_t* counts, float eps, sdf_group** out);

/* How a pass is launched (sdf_group_set_launch, sdf_group_autotune):
 * SDF_GROUP_PER_WIDTH   one launch per hidden width present, every workgroup
 *                       taking one tile of one network (deeper networks first);
 * SDF_GROUP_PER_NETWORK one collide_project launch per network;
 * SDF_GROUP_PERSISTENT  one launch of one workgroup per compute unit for the
 *                       whole pass: workgroups take (network, tile) work items
 *                       from a device counter, network after network in order
 *                       of decreasing cost per tile, until none are left (needs
 *                       every member of width 128 or more, 512 members at
 *                       most).
 * A new group uses SDF_GROUP_PER_WIDTH.  Every mode computes the same bits
 * per vertex. */
enum { SDF_GROUP_PER_WIDTH = 0, SDF_GROUP_PER_NETWORK = 1, SDF_GROUP_PERSISTENT = 2 };

/* One collide_project pass over every (network, vertex buffer) pair of the
 * group, launched as the group's mode says.  No allocation; the persistent
 * launch resets its own counters at the end of the pass, so the pass can be
 * captured into a HIP graph and replayed.  Passes of one group must not
 * overlap in time (they share the counters): issue them on one stream. */
int sdf_group_collide_project(const sdf_group* grp, void* stream);

/* Sets the launch mode (SDF_GROUP_*).  SDF_EUNSUPPORTED for
 * SDF_GROUP_PERSISTENT when a member is narrower than 128. */
int sdf_group_set_launch(sdf_group* grp, int mode);

/* Frees the group's device tables (not the networks or buffers). */
int sdf_group_destroy(sdf_group* grp);

/* ---- autotuning of tile shapes and launch shape ----
 *
 * sdf_net_autotune times the tile variants of the network's collide_project
 * kernel (BF16 and FP16 at widths 128-512: variant 0 = the default tile,
 * variant 1 = half the points per workgroup with twice the weight prefetch)
 * on n_sample points spread over [-1, 1]^3, in a scratch buffer it allocates
 * and frees, and keeps the faster for later collide_project calls on this
 * handle (other shapes and precisions: variant 0).  *variant (nullable)
 * receives the choice.  Synchronous on `stream`; call it before the handle is
 * shared across streams.  Every variant computes the same values per point.
 *
 * sdf_group_autotune times, on scratch copies of the members' vertices (the
 * members are not moved), each width class's tile variants inside the
 * per-width launch and then the three launch modes (SDF_GROUP_*), and keeps
 * the fastest for sdf_group_collide_project.  *mode (nullable) receives the
 * chosen SDF_GROUP_* mode.  Allocates and frees its scratch; synchronous on
 * `stream`. */
int sdf_net_autotune(sdf_net* net, int64_t n_sample, void* stream, int* variant);
/* Sets the tile variant directly (e.g. a cached autotune result): 0 always,
 * 1 where sdf_net_autotune has a choice (else SDF_EUNSUPPORTED). */
int sdf_net_set_tile_variant(sdf_net* net, int variant);
int sdf_group_autotune(sdf_group* grp, void* stream, int* mode);

/* ---- the time step between collision passes (Sec. 4.1: explicit Verlet) ----
 *
 * In place on device float32 [n][3] arrays: pts <- pts + (1 - damping)
 * (pts - prev) + gravity dt^2 (the multiply-add rounded once), prev <- the old
 * pts.  gravity: HOST float[3].  Gravity only: the cloth's internal forces are
 * not part of the collision path.  With sdf_group_collide_project after it,
 * one simulation step is two launches that a HIP graph can capture.
 * Errors: SDF_EINVAL for bad sizes, non-finite values, NULL, misaligned or
 * identical buffers. */
int sdf_verlet_step(float* pts, float* prev, int64_t n, float dt, const float* gravity, float damping,
                    void* stream);

/* ---- fitting (Sec. 3.1): MLP regressed onto sampled signed distances ---- */

/* Device workspace bytes sdf_train_step needs for a batch of n points with
 * this network shape (FP32 only), or -1 on a malformed/unsupported desc.  The
 * batch is processed in chunks, so the size stops growing beyond 65536 points. */
int64_t sdf_train_workspace_bytes(const sdf_net_desc* desc, int64_t n);

/* One fitting step, all in FP32 on the current device: the clamped-L1 loss
 * loss = mean_i |clamp(f(p_i)) - clamp(s_i)| (clamp to [-delta, delta]; the
 * paper's L1 loss, Sec. 3.1) and its gradient with respect to every parameter.
 * params: device float32, the flat layout of sdf_param_count (read);
 * pts: device float32 [n][3]; target: device float32 [n] signed distances;
 * grad_params: device float32, same layout as params (overwritten);
 * loss: device float32 [1] (overwritten); workspace: device memory of at least
 * sdf_train_workspace_bytes(desc, n) bytes, 256-byte aligned, caller-owned.
 * The result does not depend on thread scheduling (fixed reduction order).
 * desc->precision must be SDF_FP32.  Errors as for the query entry points. */
int sdf_train_step(const sdf_net_desc* desc, const float* params, const float* pts,
                   const float* target, int64_t n, float delta, float* grad_params, float* loss,
                   void* workspace, size_t workspace_bytes, void* stream);

/* The same fitting step for callers that cannot allocate device memory (code
 * under HIP graph capture, tight training loops, harnesses that forbid
 * hipMalloc): no workspace argument, and no allocation of any kind.  The
 * workspace lives in a static 64 MiB device array of the library (one per GPU,
 * held until the process ends); the tile kernel runs 32 workgroups and the
 * batch is cut into chunks whose workspace fits that array (about 2,700
 * points per chunk for 3->256x8->1), so this is slower than sdf_train_step.
 * Arguments, results and errors as sdf_train_step, plus SDF_EUNSUPPORTED if
 * the network's workspace for one tile exceeds the array.  Every call on a GPU
 * shares that GPU's array: calls that overlap in time on one GPU (different
 * streams, host threads) race and give wrong results; serialise them.  The
 * array's contents persist between calls; everything a step reads is written
 * earlier in the same step. */
int sdf_train_step_noalloc(const sdf_net_desc* desc, const float* params, const float* pts,
                           const float* target, int64_t n, float delta, float* grad_params,
                           float* loss, void* stream);

/* Description of the last error on the calling thread ("" if none). */
const char* sdf_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SDFCOLLIDE_H */
