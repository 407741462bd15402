// Parameter update of the mapping stage: the per-Gaussian gradients of the
// preprocessing backward (Step 5) update the 3D Gaussian parameters (Sec. 3.1).
// The paper does not name the optimiser; this is Adam without weight decay,
// the rule 3DGS-style mapping uses, for every parameter tensor of one or many
// sessions in a single launch.
//
// Per element, with t the step count after this update:
//   m <- beta1 m + (1 - beta1) g
//   v <- beta2 v + (1 - beta2) g^2
//   p <- p - (lr / (1 - beta1^t)) m / (sqrt(v) / sqrt(1 - beta2^t) + eps)
// The two bias factors are formed on the host in double precision.  Pure
// streaming work (28 bytes per element): 16-byte vector accesses, one
// block per 1024 elements of a tensor.
#include "rtgs_internal.h"

namespace rtgs {
namespace {

static_assert(sizeof(AdamArgs) <= 4000, "Adam launch table must fit the kernel arguments");

__device__ __forceinline__ void adam_one(float& p, float g, float& m, float& v,
                                         const AdamArgs& a, float step, float isb2) {
  adam_update(p, g, m, v, a.beta1, a.beta2, a.omb1, a.omb2, a.eps, step, isb2);
}

__global__ __launch_bounds__(256) void k_adam(AdamArgs a) {
  // group of this block: last group whose first block is <= blockIdx.x
  int lo = 0, hi = a.n_groups - 1;
  const int b = (int)blockIdx.x;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (a.grp[mid].block0 <= b) lo = mid;
    else hi = mid - 1;
  }
  const AdamGroupDev& G = a.grp[lo];
  const int64_t i0 = ((int64_t)(b - G.block0) * 256 + threadIdx.x) * kAdamPerThread;
  if (i0 >= G.n) return;
  if (G.vec && i0 + kAdamPerThread <= G.n) {
    float4 p = *reinterpret_cast<const float4*>(G.p + i0);
    const float4 g = *reinterpret_cast<const float4*>(G.g + i0);
    float4 m = *reinterpret_cast<const float4*>(G.m + i0);
    float4 v = *reinterpret_cast<const float4*>(G.v + i0);
    adam_one(p.x, g.x, m.x, v.x, a, G.step_size, G.inv_sqrt_bc2);
    adam_one(p.y, g.y, m.y, v.y, a, G.step_size, G.inv_sqrt_bc2);
    adam_one(p.z, g.z, m.z, v.z, a, G.step_size, G.inv_sqrt_bc2);
    adam_one(p.w, g.w, m.w, v.w, a, G.step_size, G.inv_sqrt_bc2);
    *reinterpret_cast<float4*>(G.p + i0) = p;
    *reinterpret_cast<float4*>(G.m + i0) = m;
    *reinterpret_cast<float4*>(G.v + i0) = v;
    return;
  }
  const int64_t i1 = i0 + kAdamPerThread < G.n ? i0 + kAdamPerThread : G.n;
  for (int64_t i = i0; i < i1; ++i) {
    float p = G.p[i], m = G.m[i], v = G.v[i];
    adam_one(p, G.g[i], m, v, a, G.step_size, G.inv_sqrt_bc2);
    G.p[i] = p;
    G.m[i] = m;
    G.v[i] = v;
  }
}

}  // namespace

hipError_t launch_adam(const AdamArgs& a, hipStream_t st, StageTimer* tm) {
  if (a.n_blocks <= 0) return hipSuccess;
  Scope sc(tm, kStAdam, st);
  k_adam<<<a.n_blocks, 256, 0, st>>>(a);
  return hipGetLastError();
}

}  // namespace rtgs
