// sdf_step.hip -- the time step that drives collision passes in a cloth
// simulation: the paper's simulator integrates with explicit Verlet (Sec.
// 4.1), here under gravity alone (the cloth's internal forces are not part of
// the collision path):
//   x_{t+1} = x_t + k (x_t - x_{t-1}) + g dt^2,   k = 1 - damping,
//   x_{t-1} <- x_t.
// Flat float view of the [n][3] vertex arrays: element e is component e % 3,
// so every load and store is coalesced.
#include "sdf_device.hpp"

namespace sdfc {

__global__ void __launch_bounds__(256) verlet_kernel(float* __restrict__ x, float* __restrict__ xp,
                                                     int64_t m, float k, float c0, float c1, float c2) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x) {
    const float xi = x[e], pi = xp[e];
    const int c = (int)(e % 3);
    const float gc = c == 0 ? c0 : (c == 1 ? c1 : c2);
    x[e] = __builtin_fmaf(k, xi - pi, xi) + gc;
    xp[e] = xi;
  }
}

}  // namespace sdfc
