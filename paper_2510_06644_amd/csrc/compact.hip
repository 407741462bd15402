// The mask-prune schedule of Sec. 4.1 (Adaptive Gaussian Pruning): Gaussians
// masked for K iterations are then permanently removed (stable compaction of
// every per-Gaussian array), and the next interval K follows the change ratio
// of tile-Gaussian intersections over the interval.
#include <mutex>

#include "rtgs_internal.h"

namespace rtgs {

// Scratch of the allocation-free compaction (compact_by_mask_static): the
// per-block kept counts, one word per kCompactBlock rows plus one, so at most
// (kCompactStaticWords - 1) * kCompactBlock rows.  A file-scope device array:
// every GPU the library runs on holds its own copy until the process ends.
// In host code `scratch` names a host-side stand-in; kernels get the device
// address that hipGetSymbolAddress returns for the current GPU.
static __device__ __align__(256) uint32_t scratch[kCompactStaticWords];

namespace {

static_assert(sizeof(CompactArgs) <= 4000, "compaction table must fit the kernel arguments");

// Kept count of each block of kCompactBlock rows.
__global__ __launch_bounds__(kCompactBlock) void k_compact_count(CompactArgs a) {
  __shared__ uint32_t s_w[kCompactBlock / 64];
  const int i = blockIdx.x * kCompactBlock + threadIdx.x;
  const bool keep = i < a.n && a.drop[i] == 0;
  const unsigned long long b = __ballot(keep);
  if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = (uint32_t)__popcll(b);
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (int w = 0; w < kCompactBlock / 64; ++w) t += s_w[w];
    a.block_keep[blockIdx.x] = t;
  }
}

// Exclusive scan of the block counts (one workgroup); the total is n_kept.
__global__ __launch_bounds__(kCompactBlock) void k_compact_scan(CompactArgs a, int nb) {
  __shared__ uint32_t s_part[kCompactBlock];
  // each thread scans a contiguous run of blocks
  const int per = (nb + kCompactBlock - 1) / kCompactBlock;
  const int b0 = threadIdx.x * per, b1 = min(b0 + per, nb);
  uint32_t sum = 0;
  for (int b = b0; b < b1; ++b) sum += a.block_keep[b];
  s_part[threadIdx.x] = sum;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t run = 0;
    for (int t = 0; t < kCompactBlock; ++t) {
      const uint32_t x = s_part[t];
      s_part[t] = run;
      run += x;
    }
    *a.n_kept = (int32_t)run;
  }
  __syncthreads();
  uint32_t run = s_part[threadIdx.x];
  for (int b = b0; b < b1; ++b) {
    const uint32_t x = a.block_keep[b];
    a.block_keep[b] = run;
    run += x;
  }
}

// Row i goes to position (block offset + kept rows before it in the block).
__global__ __launch_bounds__(kCompactBlock) void k_compact_scatter(CompactArgs a) {
  __shared__ uint32_t s_w[kCompactBlock / 64];
  const int i = blockIdx.x * kCompactBlock + threadIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const bool keep = i < a.n && a.drop[i] == 0;
  const unsigned long long b = __ballot(keep);
  if (lane == 0) s_w[wave] = (uint32_t)__popcll(b);
  __syncthreads();
  if (!keep) return;
  uint32_t pos = a.block_keep[blockIdx.x];
  for (int w = 0; w < wave; ++w) pos += s_w[w];
  pos += (uint32_t)__popcll(b & ((1ull << lane) - 1ull));
  for (int k = 0; k < a.n_items; ++k) {
    const CompactItemDev& it = a.item[k];
    if ((int64_t)pos >= it.dst_rows) continue;
    const int rb = it.row_bytes;
    const unsigned char* src = it.src + (int64_t)i * rb;
    unsigned char* dst = it.dst + (int64_t)pos * rb;
    if ((rb & 3) == 0) {
      for (int q = 0; q < rb; q += 4)
        *reinterpret_cast<uint32_t*>(dst + q) = *reinterpret_cast<const uint32_t*>(src + q);
    } else {
      for (int q = 0; q < rb; ++q) dst[q] = src[q];
    }
  }
}

// Tiles of a rectangle (x0, y0, x1, y1), inclusive; empty when x1 < x0.
__device__ __forceinline__ int64_t rect_area(int4 r) {
  return r.z < r.x || r.w < r.y ? 0 : (int64_t)(r.z - r.x + 1) * (r.w - r.y + 1);
}

// out[0] = sum over Gaussians not skipped of |A xor B| (tiles in exactly one
// of the two rectangles), out[1] = sum of |A|.  One workgroup, fixed order.
__global__ __launch_bounds__(kCompactBlock) void k_rect_change(const int4* A, const int4* Bv,
                                                               const uint8_t* skip, int n,
                                                               int64_t* out) {
  __shared__ long long s_d[kCompactBlock], s_r[kCompactBlock];
  long long d = 0, r = 0;
  for (int i = threadIdx.x; i < n; i += kCompactBlock) {
    if (skip && skip[i]) continue;
    const int4 a = A[i], b = Bv[i];
    const int4 c = make_int4(max(a.x, b.x), max(a.y, b.y), min(a.z, b.z), min(a.w, b.w));
    const int64_t na = rect_area(a), nb = rect_area(b), nc = rect_area(c);
    d += na + nb - 2 * nc;
    r += na;
  }
  s_d[threadIdx.x] = d;
  s_r[threadIdx.x] = r;
  __syncthreads();
  for (int w = kCompactBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      s_d[threadIdx.x] += s_d[threadIdx.x + w];
      s_r[threadIdx.x] += s_r[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = s_d[0];
    out[1] = s_r[0];
  }
}

}  // namespace

hipError_t launch_compact(const CompactArgs& a, hipStream_t st) {
  const int nb = (a.n + kCompactBlock - 1) / kCompactBlock;
  if (nb == 0) {
    k_compact_scan<<<1, kCompactBlock, 0, st>>>(a, 0);
    return hipGetLastError();
  }
  k_compact_count<<<nb, kCompactBlock, 0, st>>>(a);
  k_compact_scan<<<1, kCompactBlock, 0, st>>>(a, nb);
  k_compact_scatter<<<nb, kCompactBlock, 0, st>>>(a);
  return hipGetLastError();
}

hipError_t compact_static_scratch(uint32_t** out) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static uint32_t* ptr[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!ptr[dev]) {
    // once per device, with that device current
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    ptr[dev] = static_cast<uint32_t*>(p);
  }
  *out = ptr[dev];
  return hipSuccess;
}

hipError_t launch_rect_change(const int32_t* a, const int32_t* b, const uint8_t* skip, int n,
                              int64_t* out, hipStream_t st) {
  k_rect_change<<<1, kCompactBlock, 0, st>>>(reinterpret_cast<const int4*>(a),
                                             reinterpret_cast<const int4*>(b), skip, n, out);
  return hipGetLastError();
}

}  // namespace rtgs
