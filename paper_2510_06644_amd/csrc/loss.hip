// Gradient of the photometric + geometric loss (Eq. 6) with respect to the
// rendered colour and depth: L1 colour plus lambda_d times L1 depth, each a
// mean over the active pixels.  One pass over the frame, one pixel per
// thread (coalesced planes); the active-pixel count may come from the
// device (the count of a downsampling mask), so no host round trip is
// needed.
#include "rtgs_internal.h"

namespace rtgs {
namespace {

static_assert(sizeof(LossBatchArgs) <= 4000, "loss table must fit the kernel arguments");

__device__ __forceinline__ void l1_grad_pixel(const LossArgs& a, int64_t p) {
  const int64_t hw = (int64_t)a.w * a.h;
  if (p >= hw) return;
  const float n = a.n_active ? fmaxf((float)*a.n_active, 1.f) : (float)hw;
  const float sc = a.w_color / (3.f * n), sd = a.w_depth / n;
  const float m = a.mask ? (a.mask[p] ? 1.f : 0.f) : 1.f;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const int64_t q = c * hw + p;
    a.g_color[q] = m * sc * sign_of(a.color[q] - a.t_color[q]);
  }
  a.g_depth[p] = m * sd * sign_of(a.depth[p] - a.t_depth[p]);
}

__global__ __launch_bounds__(256) void k_l1_grad(LossArgs a) {
  l1_grad_pixel(a, (int64_t)blockIdx.x * 256 + threadIdx.x);
}

// Block b belongs to the last item whose block_base <= b.
__global__ __launch_bounds__(256) void k_l1_grad_batched(LossBatchArgs a) {
  int lo = 0, hi = a.n - 1;
  const int b = (int)blockIdx.x;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (a.item[mid].block_base <= b) lo = mid;
    else hi = mid - 1;
  }
  const LossItemDev& it = a.item[lo];
  l1_grad_pixel(it.a, (int64_t)(b - it.block_base) * 256 + threadIdx.x);
}

}  // namespace

hipError_t launch_l1_grad(const LossArgs& a, hipStream_t st) {
  const int64_t hw = (int64_t)a.w * a.h;
  if (hw <= 0) return hipSuccess;
  const int64_t blocks = (hw + 255) / 256;
  k_l1_grad<<<(unsigned)blocks, 256, 0, st>>>(a);
  return hipGetLastError();
}

hipError_t launch_l1_grad_batched(const LossBatchArgs& a, int total_blocks, hipStream_t st) {
  if (a.n <= 0 || total_blocks <= 0) return hipSuccess;
  k_l1_grad_batched<<<(unsigned)total_blocks, 256, 0, st>>>(a);
  return hipGetLastError();
}

}  // namespace rtgs
