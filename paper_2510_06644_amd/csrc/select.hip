// The two redundancy reductions of Sec. 4 as device-side selections.
//
// prune_by_grad (Sec. 4.1, Eq. 7): importance = ||dL/dmu|| + lambda ||dL/dSigma||_F
// per Gaussian (float64, rounded to float32), then the floor(ratio V) lowest
// (score, index) among visible, unmasked Gaussians join the mask.  The k-th
// smallest score is found by a 4-pass 8-bit radix select over the float bits
// (scores are >= 0, so bit order is value order), ties at the threshold go to
// the lowest indices through a block scan.  Everything stays on the device;
// a 16 KB scratch owned by the handle holds histograms and block counts.
//
// downsample_mask (Sec. 4.2): one thread per block of 2^ceil(j/2) x
// 2^floor(j/2) pixels keeps the pixel with the lowest previous final T.
#include "rtgs_internal.h"

namespace rtgs {
namespace {

constexpr int kHist = 0;          // 256 bins
constexpr int kState = 256;       // [0] V, [1] k, [2] prefix, [3] rank, [4] done flag
constexpr int kBlockCnt = 512;    // per-block equal counts (exclusive prefix after scan)
constexpr int kSelBlocks = 2048;  // max blocks of the final passes
constexpr int kSelThreads = 1024;

__device__ __forceinline__ bool candidate(const uint8_t* vis, const uint8_t* mask, int i) {
  return (vis == nullptr || vis[i] != 0) && (mask == nullptr || mask[i] == 0);
}

__device__ __forceinline__ uint32_t score_bits(const float* gm, const float* gc, float lam, int i) {
  const double a = gm[3 * i], b = gm[3 * i + 1], c = gm[3 * i + 2];
  const double xx = gc[6 * i], xy = gc[6 * i + 1], xz = gc[6 * i + 2];
  const double yy = gc[6 * i + 3], yz = gc[6 * i + 4], zz = gc[6 * i + 5];
  const double fro = sqrt(xx * xx + yy * yy + zz * zz + 2.0 * (xy * xy + xz * xz + yz * yz));
  const float s = (float)(sqrt(a * a + b * b + c * c) + (double)lam * fro);
  return __float_as_uint(s);
}

__global__ void k_prune_init(uint32_t* scr) {
  const int i = threadIdx.x;
  if (i < 256) scr[kHist + i] = 0;
  if (i < 8) scr[kState + i] = 0;
}

__global__ void k_prune_count(const uint8_t* vis, const uint8_t* mask, int n, uint32_t* scr) {
  __shared__ uint32_t c;
  if (threadIdx.x == 0) c = 0;
  __syncthreads();
  uint32_t mine = 0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    mine += candidate(vis, mask, i) ? 1u : 0u;
  atomicAdd(&c, mine);
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(&scr[kState + 0], c);
}

__global__ void k_prune_setup(uint32_t* scr, float ratio, int* n_masked) {
  const uint32_t v = scr[kState + 0];
  const uint32_t k = (uint32_t)floor((double)ratio * (double)v);
  scr[kState + 1] = k;
  scr[kState + 2] = 0;     // prefix
  scr[kState + 3] = k;     // rank still to place (1-based while searching)
  if (n_masked) *n_masked = (int)k;
}

// Histogram of the 8-bit digit at `shift` among candidates whose higher bits
// equal the current prefix.
__global__ void k_prune_hist(const float* gm, const float* gc, float lam, const uint8_t* vis,
                             const uint8_t* mask, int n, int shift, uint32_t* scr) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const uint32_t prefix = scr[kState + 2];
  const bool active = scr[kState + 3] > 0;
  if (active) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
      if (!candidate(vis, mask, i)) continue;
      const uint32_t key = score_bits(gm, gc, lam, i);
      const uint32_t hiBits = shift == 24 ? 0u : (key >> (shift + 8));
      if (hiBits != (shift == 24 ? 0u : prefix)) continue;
      atomicAdd(&h[(key >> shift) & 255u], 1u);
    }
  }
  __syncthreads();
  if (h[threadIdx.x]) atomicAdd(&scr[kHist + threadIdx.x], h[threadIdx.x]);
}

// Pick the digit holding the remaining rank; extend the prefix; clear bins.
__global__ void k_prune_pick(uint32_t* scr) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = scr[kHist + threadIdx.x];
  scr[kHist + threadIdx.x] = 0;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t r = scr[kState + 3];
    if (r > 0) {
      uint32_t d = 0;
      while (d < 255 && h[d] < r) { r -= h[d]; ++d; }
      scr[kState + 2] = (scr[kState + 2] << 8) | d;
      scr[kState + 3] = r;     // rank among keys equal to the final prefix
    }
  }
}

__device__ __forceinline__ int sel_chunk(int n, int nb) {
  const int per = (n + nb - 1) / nb;
  return ((per + kSelThreads - 1) / kSelThreads) * kSelThreads;
}

// Per-block count of candidates whose key equals the threshold.
__global__ __launch_bounds__(kSelThreads) void k_prune_eqcount(const float* gm, const float* gc,
                                                              float lam, const uint8_t* vis,
                                                              const uint8_t* mask, int n, int nb,
                                                              uint32_t* scr) {
  __shared__ uint32_t c;
  if (threadIdx.x == 0) c = 0;
  __syncthreads();
  const uint32_t tau = scr[kState + 2];
  const bool any = scr[kState + 1] > 0;
  const int chunk = sel_chunk(n, nb);
  const int beg = blockIdx.x * chunk, end = min(n, beg + chunk);
  uint32_t mine = 0;
  if (any)
    for (int i = beg + threadIdx.x; i < end; i += kSelThreads)
      mine += (candidate(vis, mask, i) && score_bits(gm, gc, lam, i) == tau) ? 1u : 0u;
  atomicAdd(&c, mine);
  __syncthreads();
  if (threadIdx.x == 0) scr[kBlockCnt + blockIdx.x] = c;
}

__global__ void k_prune_scan(uint32_t* scr, int nb) {
  if (threadIdx.x == 0) {
    uint32_t run = 0;
    for (int b = 0; b < nb; ++b) {
      const uint32_t c = scr[kBlockCnt + b];
      scr[kBlockCnt + b] = run;
      run += c;
    }
  }
}

__global__ __launch_bounds__(kSelThreads) void k_prune_final(const float* gm, const float* gc,
                                                            float lam, const uint8_t* vis,
                                                            const uint8_t* mask_in, int n, int nb,
                                                            uint32_t* scr, uint8_t* mask_out,
                                                            float* score_out) {
  __shared__ uint32_t wsum[kSelThreads / 64];
  const uint32_t tau = scr[kState + 2];
  const uint32_t take = scr[kState + 3];
  const bool any = scr[kState + 1] > 0;
  const int chunk = sel_chunk(n, nb);
  const int beg = blockIdx.x * chunk, end = min(n, beg + chunk);
  uint32_t run = scr[kBlockCnt + blockIdx.x];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int base = beg; base < end; base += kSelThreads) {
    const int i = base + threadIdx.x;
    bool cand = false, eq = false, lt = false;
    uint32_t key = 0;
    if (i < end) {
      cand = candidate(vis, mask_in, i);
      key = score_bits(gm, gc, lam, i);
      if (score_out) score_out[i] = __uint_as_float(key);
      eq = cand && key == tau;
      lt = cand && key < tau;
    }
    const unsigned long long bal = __ballot(eq);
    const uint32_t before_in_wave = __popcll(bal & ((1ull << lane) - 1ull));
    if (lane == 0) wsum[wave] = (uint32_t)__popcll(bal);
    __syncthreads();
    uint32_t before = run + before_in_wave;
    for (int q = 0; q < wave; ++q) before += wsum[q];
    uint32_t tot = 0;
    for (int q = 0; q < kSelThreads / 64; ++q) tot += wsum[q];
    __syncthreads();
    if (i < end) {
      const bool sel = any && (lt || (eq && before < take));
      const bool was = mask_in != nullptr && mask_in[i] != 0;
      mask_out[i] = (was || sel) ? 1 : 0;
    }
    run += tot;
  }
}

__global__ void k_ds_init(int* n_active) {
  if (threadIdx.x == 0 && n_active) *n_active = 0;
}

__global__ void k_downsample(const float* T, int w, int h, int bw, int bh, uint8_t* mask,
                             int* n_active) {
  const int nbx = (w + bw - 1) / bw, nby = (h + bh - 1) / bh;
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nbx * nby) return;
  const int x0 = (b % nbx) * bw, y0 = (b / nbx) * bh;
  const int x1 = min(w, x0 + bw), y1 = min(h, y0 + bh);
  int best = y0 * w + x0;
  float bt = T[best];
  for (int y = y0; y < y1; ++y)
    for (int x = x0; x < x1; ++x) {
      const int p = y * w + x;
      const float t = T[p];
      if (t < bt) { bt = t; best = p; }       // row-major visit: first minimum wins
    }
  for (int y = y0; y < y1; ++y)
    for (int x = x0; x < x1; ++x) mask[y * w + x] = (y * w + x == best) ? 1 : 0;
  if (n_active) atomicAdd(n_active, 1);
}

}  // namespace

hipError_t launch_prune(const float* g_means, const float* g_cov3d, const uint8_t* visible,
                        const uint8_t* mask_in, int n, float lambda, float ratio,
                        uint8_t* mask_out, int* n_masked, float* score_out, uint32_t* scr,
                        hipStream_t st) {
  k_prune_init<<<1, 256, 0, st>>>(scr);
  if (n <= 0) {
    k_prune_setup<<<1, 1, 0, st>>>(scr, ratio, n_masked);
    return hipGetLastError();
  }
  const int grid = min(1024, (n + 255) / 256);
  k_prune_count<<<grid, 256, 0, st>>>(visible, mask_in, n, scr);
  k_prune_setup<<<1, 1, 0, st>>>(scr, ratio, n_masked);
  for (int shift = 24; shift >= 0; shift -= 8) {
    k_prune_hist<<<grid, 256, 0, st>>>(g_means, g_cov3d, lambda, visible, mask_in, n, shift, scr);
    k_prune_pick<<<1, 256, 0, st>>>(scr);
  }
  const int nb = min(kSelBlocks, (n + kSelThreads - 1) / kSelThreads);
  k_prune_eqcount<<<nb, kSelThreads, 0, st>>>(g_means, g_cov3d, lambda, visible, mask_in, n, nb,
                                               scr);
  k_prune_scan<<<1, 64, 0, st>>>(scr, nb);
  k_prune_final<<<nb, kSelThreads, 0, st>>>(g_means, g_cov3d, lambda, visible, mask_in, n, nb,
                                             scr, mask_out, score_out);
  return hipGetLastError();
}

hipError_t launch_downsample(const float* final_T, int w, int h, int j, uint8_t* mask_out,
                             int* n_active, hipStream_t st) {
  const int bw = 1 << ((j + 1) / 2), bh = 1 << (j / 2);
  const int nb = ((w + bw - 1) / bw) * ((h + bh - 1) / bh);
  k_ds_init<<<1, 64, 0, st>>>(n_active);
  if (nb > 0) k_downsample<<<(nb + 255) / 256, 256, 0, st>>>(final_T, w, h, bw, bh, mask_out,
                                                            n_active);
  return hipGetLastError();
}

}  // namespace rtgs
