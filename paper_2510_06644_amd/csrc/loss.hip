// Gradient of the photometric + geometric loss (Eq. 6) with respect to the
// rendered colour and depth: L1 colour plus lambda_d times L1 depth, each a
// mean over the active pixels.  One pass over the frame, one pixel per
// thread (coalesced planes); the active-pixel count may come from the
// device (the count of a downsampling mask), so no host round trip is
// needed.
#include "rtgs_internal.h"

namespace rtgs {
namespace {

__device__ __forceinline__ float sgn(float x) { return x > 0.f ? 1.f : (x < 0.f ? -1.f : 0.f); }

__global__ __launch_bounds__(256) void k_l1_grad(LossArgs a) {
  const int64_t hw = (int64_t)a.w * a.h;
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= hw) return;
  const float n = a.n_active ? fmaxf((float)*a.n_active, 1.f) : (float)hw;
  const float sc = a.w_color / (3.f * n), sd = a.w_depth / n;
  const float m = a.mask ? (a.mask[p] ? 1.f : 0.f) : 1.f;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const int64_t q = c * hw + p;
    a.g_color[q] = m * sc * sgn(a.color[q] - a.t_color[q]);
  }
  a.g_depth[p] = m * sd * sgn(a.depth[p] - a.t_depth[p]);
}

}  // namespace

hipError_t launch_l1_grad(const LossArgs& a, hipStream_t st) {
  const int64_t hw = (int64_t)a.w * a.h;
  if (hw <= 0) return hipSuccess;
  const int64_t blocks = (hw + 255) / 256;
  k_l1_grad<<<(unsigned)blocks, 256, 0, st>>>(a);
  return hipGetLastError();
}

}  // namespace rtgs
