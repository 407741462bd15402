// Steps 1 and 2 of the forward pass (Sec. 2.1): projection of every Gaussian
// (Step 1-1), tile intersection (Step 1-2) and per-tile depth sorting
// (Step 2), for a batch of sessions sharing one tile space.
//
// Design for gfx950:
//  * projection runs one thread per Gaussian in float64: it is HBM bound
//    (56 B in, 64 B out per Gaussian), and float64 lets the raster kernels see
//    pixel-space centres split as hi + lo float32 parts, so their float32
//    compositing matches the float64 definition far below 1e-4;
//  * binning is a counting sort by tile without global atomics (device-scope
//    atomics cross the XCDs and serialise).  Each workgroup takes a chunk of
//    1024 Gaussians and counts its (tile, Gaussian) pairs per tile in an LDS
//    histogram.  Column sums over the chunks give each tile's list length and
//    start.  A second pass over the chunk orders its pairs by tile in LDS
//    and writes them as one contiguous block (chunk-major: every store is
//    coalesced, where scattering 8-byte keys into the tile ranges made the
//    memory system merge millions of partial lines).  One workgroup per tile
//    then gathers the tile's run from every chunk and sorts it in LDS (merge
//    sort of 64-bit keys; long lists are gathered to global memory and go to
//    a second kernel with 1024 threads, sorting in place beyond its LDS).
//    The same pass writes each Gaussian's first slot in Gaussian-major pair
//    order, which the backward uses to merge gradients without atomics.  No
//    host sync: the pair total stays on the device, and a capacity overflow
//    publishes empty tile lists (every list entry is always a real pair).
#include "rtgs_internal.h"

namespace rtgs {
namespace {

constexpr int kScanThreads = 1024;

__global__ void k_init(long long* counters) {
  if (threadIdx.x < 8) counters[threadIdx.x] = 0;
}

struct Proj {
  double u, v, z, sxx, sxy, syy;
  bool ok;
};

// Step 1-1 for one Gaussian in float64 (EWA, first order).
__device__ __forceinline__ void project_one(const SessionDev& S, const float* vm, int li,
                                            double& o, Proj& P) {
  const double mx = S.means[3 * li + 0], my = S.means[3 * li + 1], mz = S.means[3 * li + 2];
  const double qw = S.quats[4 * li + 0], qx = S.quats[4 * li + 1];
  const double qy = S.quats[4 * li + 2], qz = S.quats[4 * li + 3];
  double ss[3];
  activate(S, li, ss, o);
  P.ok = false;
  // camera-space centre p = R_c mu + t_c
  const double x = vm[0] * mx + vm[1] * my + vm[2] * mz + vm[3];
  const double y = vm[4] * mx + vm[5] * my + vm[6] * mz + vm[7];
  const double z = vm[8] * mx + vm[9] * my + vm[10] * mz + vm[11];
  P.z = z;
  if (!(z > kNearZ) || !(255.0 * o >= 1.0)) return;
  if (S.gmask && S.gmask[li]) return;
  // rotation of the normalised quaternion (w, x, y, z)
  const double qn = 1.0 / sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
  const double w = qw * qn, a = qx * qn, b = qy * qn, c = qz * qn;
  double R[9] = {1 - 2 * (b * b + c * c), 2 * (a * b - w * c), 2 * (a * c + w * b),
                 2 * (a * b + w * c), 1 - 2 * (a * a + c * c), 2 * (b * c - w * a),
                 2 * (a * c - w * b), 2 * (b * c + w * a), 1 - 2 * (a * a + b * b)};
  // M = R diag(s); Sigma = M M^T
  double M[9];
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < 3; ++k) M[3 * r + k] = R[3 * r + k] * ss[k];
  // EWA Jacobian with the field-of-view clamp
  const double limx = kFovClamp * 0.5 * S.width / S.fx;
  const double limy = kFovClamp * 0.5 * S.height / S.fy;
  const double iz = 1.0 / z;      // once: a float64 division is a long instruction sequence
  const double rx = x * iz, ry = y * iz;
  const double tx = fmin(limx, fmax(-limx, rx));
  const double ty = fmin(limy, fmax(-limy, ry));
  const double j00 = S.fx * iz, j02 = -S.fx * tx * iz;
  const double j11 = S.fy * iz, j12 = -S.fy * ty * iz;
  // T = J W (2x3), W = R_c
  double T0[3], T1[3];
  for (int k = 0; k < 3; ++k) {
    T0[k] = j00 * vm[0 + k] + j02 * vm[8 + k];
    T1[k] = j11 * vm[4 + k] + j12 * vm[8 + k];
  }
  // A = T M (2x3); Sigma' = A A^T + dilation
  double A0[3], A1[3];
  for (int k = 0; k < 3; ++k) {
    A0[k] = T0[0] * M[0 + k] + T0[1] * M[3 + k] + T0[2] * M[6 + k];
    A1[k] = T1[0] * M[0 + k] + T1[1] * M[3 + k] + T1[2] * M[6 + k];
  }
  P.sxx = A0[0] * A0[0] + A0[1] * A0[1] + A0[2] * A0[2] + kDilation;
  P.sxy = A0[0] * A1[0] + A0[1] * A1[1] + A0[2] * A1[2];
  P.syy = A1[0] * A1[0] + A1[1] * A1[1] + A1[2] * A1[2] + kDilation;
  P.u = S.fx * rx + S.cx;
  P.v = S.fy * ry + S.cy;
  const double det = P.sxx * P.syy - P.sxy * P.sxy;
  P.ok = det > 0.0;
}

__device__ __forceinline__ void split(double x, float& hi, float& lo) {
  hi = (float)x;
  lo = (float)(x - (double)hi);
}

// Step 1-1 + the tile rectangle of Step 1-2 + per-tile pair counts.
// REUSE: the tile lists (and with them each Gaussian's tile rectangle, pair
// count and slots) stay those of the workspace's last full forward; only the
// raster records are recomputed for the current pose.
template <bool REUSE, bool ONE>
__global__ __launch_bounds__(kGaussPerBlock) void k_preprocess(Batch B, WsPtrs W) {
  const int s = ONE ? 0 : find_session(session_table(B), B.n_sessions, (int)blockIdx.x,
                                         [](const SessionDev& x) { return x.block_base; });
  const SessionDev& S = batch_session<ONE>(B, s);
  const int li = ((int)blockIdx.x - S.block_base) * kGaussPerBlock + (int)threadIdx.x;
  // the call's counters start at zero (the binning passes run after this kernel)
  if (!REUSE && blockIdx.x == 0 && threadIdx.x < 8) W.counters[threadIdx.x] = 0;
  if (li >= S.n) return;
  const int gid = S.gauss_base + li;
  float vm[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) vm[k] = S.viewmat[k];
  double o;
  Proj P;
  project_one(S, vm, li, o, P);
  int4 rect = make_int4(0, 0, -1, -1);
  if (P.ok) {
    const double det = P.sxx * P.syy - P.sxy * P.sxy;
    const double inv = 1.0 / det;
    float uh, ul, vh, vl;
    split(P.u, uh, ul);
    split(P.v, vh, vl);
    const float zf = (float)P.z;
    // bounding box of the alpha = 1/255 ellipse: d^T M d <= 2 ln(255 o)
    const double t = 2.0 * (double)logf((float)(255.0 * o));
    const float ex = (float)sqrt(t * P.sxx);
    const float ey = (float)sqrt(t * P.syy);
    GaussRec r;
    r.pos = make_float4(uh, vh, ul, vl);
    r.conic = make_float4((float)(P.syy * inv), (float)(-P.sxy * inv), (float)(P.sxx * inv),
                          (float)o);
    r.col = make_float4(S.colors[3 * li + 0], S.colors[3 * li + 1], S.colors[3 * li + 2], zf);
    r.ext = make_float4(ex, ey, (float)t, 0.f);
    W.rec[gid] = r;
    // padded pixel range in float32, fixed operation order (see the replay)
    const float lox = floorf((uh - ex) - 1.5f), hix = ceilf((uh + ex) + 0.5f);
    const float loy = floorf((vh - ey) - 1.5f), hiy = ceilf((vh + ey) + 0.5f);
    if (!(hix < 0.f || lox > (float)(S.width - 1) || hiy < 0.f || loy > (float)(S.height - 1))) {
      const int i0 = (int)fmaxf(lox, 0.f), i1 = (int)fminf(hix, (float)(S.width - 1));
      const int j0 = (int)fmaxf(loy, 0.f), j1 = (int)fminf(hiy, (float)(S.height - 1));
      const int shx = 4 + S.sub_sx, shy = 4 + S.sub_sy;   // tile = (16 bw) x (16 bh)
      rect = make_int4(i0 >> shx, j0 >> shy, i1 >> shx, j1 >> shy);
    }
  } else {
    GaussRec r;
    r.pos = make_float4(0.f, 0.f, 0.f, 0.f);
    r.conic = make_float4(0.f, 0.f, 0.f, 0.f);
    r.col = make_float4(0.f, 0.f, 0.f, (float)P.z);
    // a negative alpha-ellipse bound fails every quadrant test: a culled or
    // masked Gaussian left in a reused list costs the rasterizer nothing
    r.ext = make_float4(0.f, 0.f, -1.f, 0.f);
    W.rec[gid] = r;
  }
  if (REUSE) {
    const int4 ref = W.rect[gid];
    if (S.visible) S.visible[li] = ref.z >= ref.x ? 1 : 0;
    return;
  }
  W.rect[gid] = rect;
  // the depth bits of the Gaussian's sort key, read by the emit from this
  // dense array rather than from the 64-byte records
  W.zkey[gid] = __float_as_uint((float)P.z);
  const bool vis = rect.z >= rect.x;
  if (S.visible) S.visible[li] = vis ? 1 : 0;
  W.cnt[gid] = vis ? (uint32_t)((rect.z - rect.x + 1) * (rect.w - rect.y + 1)) : 0u;
}

// Threads per workgroup of the binning passes over a chunk: one Gaussian per
// thread, so the few hundred chunks of a frame still fill the chip.
constexpr int kBinThreads = 1024;
static_assert(kChunk % kBinThreads == 0, "whole rounds per chunk");

// The tile rectangles and pair counts of this thread's Gaussians of chunk c
// (local index i = j * kBinThreads + thread for round j), loaded together at
// the start of a binning pass so that their latencies overlap.
constexpr int kChunkRounds = kChunk / kBinThreads;
struct ChunkIn {
  int4 rect[kChunkRounds];
  uint32_t cnt[kChunkRounds];
};

__device__ __forceinline__ ChunkIn load_chunk(const SessionDev& S, const WsPtrs& W, int c) {
  ChunkIn in;
#pragma unroll
  for (int j = 0; j < kChunkRounds; ++j) {
    const int li = c * kChunk + j * kBinThreads + (int)threadIdx.x;
    in.rect[j] = li < S.n ? W.rect[S.gauss_base + li] : make_int4(0, 0, -1, -1);
    in.cnt[j] = li < S.n ? W.cnt[S.gauss_base + li] : 0u;
  }
  return in;
}

// The chunk's tile rectangles in LDS, so the pair walk below never waits on
// a dependent global load.  Visible after the barrier in chunk_offsets.
__device__ __forceinline__ void stage_rects(const ChunkIn& in, int4* s_rect) {
#pragma unroll
  for (int j = 0; j < kChunkRounds; ++j) s_rect[j * kBinThreads + threadIdx.x] = in.rect[j];
}

// In-chunk exclusive offsets of the Gaussians' tile counts, in local index
// order, into s_off[0..kChunk]; s_off[kChunk] = the chunk's pair total, which
// is returned.
__device__ uint32_t chunk_offsets(const ChunkIn& in, uint32_t* s_off, uint32_t* s_wave) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t carry = 0;
  for (int j = 0; j < kChunkRounds; ++j) {
    const int i = j * kBinThreads + (int)threadIdx.x;
    const uint32_t n = in.cnt[j];
    uint32_t x = n;
    for (int off = 1; off < 64; off <<= 1) {
      const uint32_t y = __shfl_up(x, off, 64);
      if (lane >= off) x += y;
    }
    if (lane == 63) s_wave[wave] = x;
    __syncthreads();
    uint32_t before = 0, tot = 0;
    for (int q = 0; q < kBinThreads / 64; ++q) {
      before += q < wave ? s_wave[q] : 0u;
      tot += s_wave[q];
    }
    s_off[i] = carry + before + x - n;
    carry += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) s_off[kChunk] = carry;
  __syncthreads();
  return carry;
}

// Walk this thread's share of the chunk's pairs: pairs [m0, m1) in
// Gaussian-major order, m0 = thread * ceil(total / kBinThreads), with the
// chunk's tile rectangles staged in LDS (s_rect[i] for local index i).  One binary search
// finds the first Gaussian; after that the walk steps through tiles of the
// Gaussian's rectangle row by row and on to the next Gaussian, so pairs are
// spread evenly however many tiles a Gaussian touches.  f(local index, tile)
// is called for every pair.
template <typename F>
__device__ __forceinline__ void chunk_pairs(const SessionDev& S, const int4* s_rect, int c,
                                            const uint32_t* s_off, uint32_t total, F f) {
  const uint32_t per = (total + kBinThreads - 1) / kBinThreads;
  const uint32_t m0 = threadIdx.x * per;
  const uint32_t m1 = min(total, m0 + per);
  if (m0 >= m1) return;
  int lo = 0, hi = kChunk - 1;          // last i with s_off[i] <= m0
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (s_off[mid] <= m0) lo = mid; else hi = mid - 1;
  }
  int i = lo;
  int4 r = s_rect[i];
  int w = r.z - r.x + 1;
  const int k0 = (int)(m0 - s_off[i]);
  int tx = r.x + k0 % w, ty = r.y + k0 / w;
  for (uint32_t m = m0; m < m1; ++m) {
    while (m >= s_off[i + 1]) {           // next Gaussian with pairs
      ++i;
      if (m < s_off[i + 1]) {
        r = s_rect[i];
        w = r.z - r.x + 1;
        tx = r.x;
        ty = r.y;
      }
    }
    f(i, ty * S.tiles_x + tx);
    if (++tx > r.z) {
      tx = r.x;
      ++ty;
    }
  }
}

// Per chunk of kChunk Gaussians: pair counts per tile of the session (LDS
// histogram), and the chunk's pair total.
template <bool ONE>
__global__ __launch_bounds__(kBinThreads) void k_chunk_hist(Batch B, WsPtrs W) {
  extern __shared__ uint32_t s_hist[];
  __shared__ uint32_t s_off[kChunk + 1];
  __shared__ int4 s_rect[kChunk];
  __shared__ uint32_t s_wave[kBinThreads / 64];
  const int s = ONE ? 0 : find_session(session_table(B), B.n_sessions, (int)blockIdx.x,
                                         [](const SessionDev& x) { return x.chunk_base; });
  const SessionDev& S = batch_session<ONE>(B, s);
  const int c = (int)blockIdx.x - S.chunk_base;
  const int ts = S.tiles_x * S.tiles_y;
  const ChunkIn in = load_chunk(S, W, c);
  for (int t = threadIdx.x; t < ts; t += kBinThreads) s_hist[t] = 0u;
  stage_rects(in, s_rect);
  const uint32_t total = chunk_offsets(in, s_off, s_wave);
  // pairs are dealt evenly over the threads, whatever the Gaussians' sizes
  chunk_pairs(S, s_rect, c, s_off, total, [&](int, int tile) { atomicAdd(&s_hist[tile], 1u); });
  __syncthreads();
  uint32_t* h = W.hist + S.hist_base + (int64_t)c * ts;
  for (int t = threadIdx.x; t < ts; t += kBinThreads) h[t] = s_hist[t];
  if (threadIdx.x == 0) W.chunk_total[blockIdx.x] = total;
}

// Column sums of the per-(chunk, tile) counts, one thread per (tile, group
// of chunks); k_scan_tiles adds the groups.
constexpr int kScanGroups = 16;

__device__ __forceinline__ void tile_groups(const SessionDev& S, int g, int& c0, int& c1) {
  const int nc = (S.n + kChunk - 1) / kChunk;
  const int per = (nc + kScanGroups - 1) / kScanGroups;
  c0 = min(nc, g * per);
  c1 = min(nc, c0 + per);
}

template <bool ONE>
__global__ __launch_bounds__(kBlock) void k_tile_group_sums(Batch B, WsPtrs W) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  const int g = blockIdx.y;
  if (t >= B.t_total) return;
  const int s = ONE ? 0 : find_session(session_table(B), B.n_sessions, t,
                                         [](const SessionDev& x) { return x.tile_base; });
  const SessionDev& S = batch_session<ONE>(B, s);
  const int ts = S.tiles_x * S.tiles_y;
  int c0, c1;
  tile_groups(S, g, c0, c1);
  const uint32_t* h = W.hist + S.hist_base + (t - S.tile_base);
  uint32_t sum = 0;
#pragma unroll 8
  for (int c = c0; c < c1; ++c) sum += h[(int64_t)c * ts];
  W.gsum[(int64_t)g * B.t_total + t] = sum;
}

// Exclusive scan of n values in[0..n) into out[0..n]; out[n] = total.  Each
// thread sums a contiguous run; the run sums are scanned inside each wave by
// lane shifts, then across the waves through LDS (part[kScanThreads / 64]),
// so two barriers in all.
__device__ uint32_t block_scan_1024(const uint32_t* in, uint32_t* out, int n, uint32_t* part) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int per = (n + kScanThreads - 1) / kScanThreads;
  const int beg = min(tid * per, n), end = min(beg + per, n);
  uint32_t sum = 0;
  for (int i = beg; i < end; ++i) sum += in[i];
  uint32_t x = sum;                       // inclusive scan of the run sums in the wave
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  if (lane == 63) part[wave] = x;
  __syncthreads();
  uint32_t before = 0, total = 0;
  for (int q = 0; q < kScanThreads / 64; ++q) {
    const uint32_t v = part[q];
    before += q < wave ? v : 0u;
    total += v;
  }
  uint32_t run = before + x - sum;
  for (int i = beg; i < end; ++i) {
    const uint32_t v = in[i];
    out[i] = run;
    run += v;
  }
  if (tid == 0) out[n] = total;
  __syncthreads();                        // part is reused by the next call
  return total;
}

// Exclusive scan across the block of the values v[0..P) that each thread
// holds for positions P tid .. P tid + P - 1; v becomes the exclusive
// prefixes, and the block total is returned.  Same two-barrier structure as
// block_scan_1024.
template <int P>
__device__ uint32_t block_scan_regs(uint32_t (&v)[P], uint32_t* part) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  uint32_t sum = 0;
#pragma unroll
  for (int i = 0; i < P; ++i) sum += v[i];
  uint32_t x = sum;
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  if (lane == 63) part[wave] = x;
  __syncthreads();
  uint32_t before = 0, total = 0;
  for (int q = 0; q < kScanThreads / 64; ++q) {
    const uint32_t w = part[q];
    before += q < wave ? w : 0u;
    total += w;
  }
  uint32_t run = before + x - sum;
#pragma unroll
  for (int i = 0; i < P; ++i) {
    const uint32_t w = v[i];
    v[i] = run;
    run += w;
  }
  __syncthreads();                        // part is reused by the next call
  return total;
}

// Tile ranges (scan of the per-tile counts, each the sum of its chunk
// groups), chunk offsets (scan of the per-chunk totals), and the pair total.
// Up to kScanPer tiles and chunks per thread the counts are loaded together
// with coalesced loads into LDS, scanned in registers (each thread a
// contiguous run) and stored coalesced from LDS: one round trip to memory.
// Larger batches scan through global memory.  When the pairs exceed the
// capacity every tile list is published empty (the call's output is invalid
// and reported, and no list holds a pair that was not stored).
constexpr int kScanPer = 4;

__global__ __launch_bounds__(kScanThreads) void k_scan_tiles(WsPtrs W, int t_total, int c_total,
                                                             unsigned long long* max_pairs) {
  __shared__ uint32_t part[kScanThreads / 64];
  __shared__ uint32_t s_t[kScanPer * kScanThreads], s_c[kScanPer * kScanThreads];
  const int tid = threadIdx.x;
  uint32_t total;
  if (t_total <= kScanPer * kScanThreads && c_total <= kScanPer * kScanThreads) {
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
      const int t = k * kScanThreads + tid;
      uint32_t sum = 0;
      if (t < t_total) {
#pragma unroll
        for (int g = 0; g < kScanGroups; ++g) sum += W.gsum[(int64_t)g * t_total + t];
      }
      s_t[t] = sum;
      s_c[t] = t < c_total ? W.chunk_total[t] : 0u;
    }
    __syncthreads();
    uint32_t tv[kScanPer], cv[kScanPer];
#pragma unroll
    for (int i = 0; i < kScanPer; ++i) {
      tv[i] = s_t[tid * kScanPer + i];
      cv[i] = s_c[tid * kScanPer + i];
    }
    total = block_scan_regs<kScanPer>(tv, part);        // its barriers order the LDS reuse
    const uint32_t ctot = block_scan_regs<kScanPer>(cv, part);
#pragma unroll
    for (int i = 0; i < kScanPer; ++i) {
      s_t[tid * kScanPer + i] = tv[i];
      s_c[tid * kScanPer + i] = cv[i];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
      const int t = k * kScanThreads + tid;
      if (t < t_total) W.tile_start[t] = s_t[t];
      if (t < c_total) W.chunk_off[t] = s_c[t];
    }
    if (tid == 0) {
      W.tile_start[t_total] = total;
      W.chunk_off[c_total] = ctot;
    }
    __syncthreads();                      // tile_start complete before an overflow clears it
  } else {
    for (int t = tid; t < t_total; t += kScanThreads) {
      uint32_t sum = 0;
#pragma unroll
      for (int g = 0; g < kScanGroups; ++g) sum += W.gsum[(int64_t)g * t_total + t];
      W.tile_count[t] = sum;
    }
    __syncthreads();
    total = block_scan_1024(W.tile_count, W.tile_start, t_total, part);
    block_scan_1024(W.chunk_total, W.chunk_off, c_total, part);
  }
  if ((int64_t)total > W.cap)
    for (int t = threadIdx.x; t <= t_total; t += kScanThreads) W.tile_start[t] = 0u;
  if (threadIdx.x == 0) {
    W.counters[0] = (long long)total;
    // [0]: largest pair count of any call; [1]: largest count of a call whose
    // capacity it exceeded (0 if none)
    atomicMax(&max_pairs[0], (unsigned long long)total);
    if ((int64_t)total > W.cap) atomicMax(&max_pairs[1], (unsigned long long)total);
  }
}

// Per chunk: each Gaussian's first Gaussian-major slot; the chunk's pairs
// ordered by tile, written as one block at chunk_off (chunk-major layout;
// inside it, tile t's run starts at the exclusive scan of the chunk's tile
// counts, which replaces the counts in this chunk's histogram row for the
// sort's gather).  The pairs are staged in LDS as 16-bit local indices and
// written with coalesced stores; a chunk with more than kStagePairs pairs
// writes them directly inside its block.
constexpr int kStagePairs = 12288;

template <bool ONE>
__global__ __launch_bounds__(kBinThreads) void k_emit(Batch B, WsPtrs W) {
  extern __shared__ uint32_t s_dyn[];       // [ts] tile cursors, then [kStagePairs] uint16
  __shared__ uint32_t s_off[kChunk + 1];
  __shared__ int4 s_rect[kChunk];
  __shared__ uint32_t s_zb[kChunk];
  __shared__ uint32_t s_wave[kBinThreads / 64];
  const int s = ONE ? 0 : find_session(session_table(B), B.n_sessions, (int)blockIdx.x,
                                         [](const SessionDev& x) { return x.chunk_base; });
  const SessionDev& S = batch_session<ONE>(B, s);
  const int c = (int)blockIdx.x - S.chunk_base;
  const int ts = S.tiles_x * S.tiles_y;
  uint32_t* s_cur = s_dyn;
  uint16_t* s_loc = reinterpret_cast<uint16_t*>(s_dyn + ts);
  uint32_t* h = W.hist + S.hist_base + (int64_t)c * ts;
  // every global load of the prologue issued together: the Gaussians' inputs,
  // their key depths and this thread's run of the chunk's tile counts
  const ChunkIn in = load_chunk(S, W, c);
  uint32_t zb[kChunkRounds];
#pragma unroll
  for (int j = 0; j < kChunkRounds; ++j) {
    const int li = c * kChunk + j * kBinThreads + (int)threadIdx.x;
    zb[j] = li < S.n ? W.zkey[S.gauss_base + li] : 0u;
  }
  constexpr int kRunMax = (kMaxTilesPerSession + kBinThreads - 1) / kBinThreads;
  const int per = (ts + kBinThreads - 1) / kBinThreads;
  const int beg = min((int)threadIdx.x * per, ts), end = min(beg + per, ts);
  uint32_t hv[kRunMax];
#pragma unroll
  for (int k = 0; k < kRunMax; ++k) hv[k] = beg + k < end ? h[beg + k] : 0u;
  // exclusive scan of the chunk's tile counts: each thread a contiguous run of
  // tiles, the run sums scanned across the waves
  {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < kRunMax; ++k) sum += hv[k];
    uint32_t x = sum;
    for (int off = 1; off < 64; off <<= 1) {
      const uint32_t y = __shfl_up(x, off, 64);
      if (lane >= off) x += y;
    }
    if (lane == 63) s_wave[wave] = x;
    __syncthreads();
    uint32_t run = x - sum;
    for (int q = 0; q < wave; ++q) run += s_wave[q];
#pragma unroll
    for (int k = 0; k < kRunMax; ++k) {
      if (beg + k < end) {
        s_cur[beg + k] = run;
        h[beg + k] = run;
      }
      run += hv[k];
    }
    __syncthreads();                        // s_wave is reused below
  }
  stage_rects(in, s_rect);
#pragma unroll
  for (int j = 0; j < kChunkRounds; ++j) s_zb[j * kBinThreads + threadIdx.x] = zb[j];
  const uint32_t total = chunk_offsets(in, s_off, s_wave);
  const uint32_t base = W.chunk_off[blockIdx.x];
  for (int j = 0; j < kChunk / kBinThreads; ++j) {
    const int i = j * kBinThreads + (int)threadIdx.x;
    const int li = c * kChunk + i;
    if (li < S.n) W.goff[S.gauss_base + li] = base + s_off[i];
  }
  const uint32_t g0 = S.gauss_base + c * kChunk;
  const bool staged = total <= kStagePairs;
  chunk_pairs(S, s_rect, c, s_off, total, [&](int i, int tile) {
    const uint32_t pos = atomicAdd(&s_cur[tile], 1u);
    if (staged)
      s_loc[pos] = (uint16_t)i;
    else if ((int64_t)base + pos < W.cap)
      W.keys[base + pos] = ((unsigned long long)s_zb[i] << 32) | (g0 + i);
  });
  if (staged) {
    __syncthreads();
    for (uint32_t k = threadIdx.x; k < total; k += kBinThreads) {
      const uint32_t i = s_loc[k];
      if ((int64_t)base + k < W.cap)
        W.keys[base + k] = ((unsigned long long)s_zb[i] << 32) | (g0 + i);
    }
  }
}

// Bitonic sorting network on a[0..n) (ascending), all merges in the "flip"
// form so that virtual +inf padding up to the next power of two never moves:
// each compare-exchange puts the minimum at the lower index, hence a pair
// whose upper index is >= n is left alone.
template <typename P>
__device__ void bitonic_sort(P a, int n) {
  int npow = 1;
  while (npow < n) npow <<= 1;
  const int half = npow >> 1;
  for (int k = 2; k <= npow; k <<= 1) {
    const int hk = k >> 1;
    for (int p = threadIdx.x; p < half; p += blockDim.x) {
      const int r = p & (hk - 1);
      const int i = (p / hk) * k + r;
      const int j = i + k - 1 - 2 * r;
      if (j < n) {
        const unsigned long long x = a[i], y = a[j];
        if (y < x) { a[i] = y; a[j] = x; }
      }
    }
    __threadfence_block();
    __syncthreads();
    for (int m = k >> 2; m >= 1; m >>= 1) {
      for (int p = threadIdx.x; p < half; p += blockDim.x) {
        const int i = (p / m) * 2 * m + (p & (m - 1));
        const int j = i + m;
        if (j < n) {
          const unsigned long long x = a[i], y = a[j];
          if (y < x) { a[i] = y; a[j] = x; }
        }
      }
      __threadfence_block();
      __syncthreads();
    }
  }
}

// Merge sort of one tile's 64-bit keys: the list is padded to N keys (a power
// of two, n <= N <= K NT) with all-ones keys, which no real key equals since
// depth bits of a finite float are below 0x7f800000.  The first N / K threads
// each sort K keys in registers, then log2(N / K) merge levels run through two
// LDS buffers: a thread finds where its K outputs start on the merge path of
// its pair of runs by binary search and merges K keys.  One barrier per level
// (all NT threads take it), instead of one per bitonic stage.
constexpr unsigned long long kKeyPad = ~0ull;
constexpr int kSortPerThread = 4;

__device__ __forceinline__ void cas(unsigned long long& a, unsigned long long& b) {
  const unsigned long long lo = a < b ? a : b, hi = a < b ? b : a;
  a = lo;
  b = hi;
}

// Sorting networks: 5 comparators for 4 keys, Batcher's 19 for 8.
__device__ __forceinline__ void sort_network(unsigned long long (&k)[4]) {
  cas(k[0], k[1]); cas(k[2], k[3]);
  cas(k[0], k[2]); cas(k[1], k[3]);
  cas(k[1], k[2]);
}
__device__ __forceinline__ void sort_network(unsigned long long (&k)[8]) {
  cas(k[0], k[1]); cas(k[2], k[3]); cas(k[4], k[5]); cas(k[6], k[7]);
  cas(k[0], k[2]); cas(k[1], k[3]); cas(k[4], k[6]); cas(k[5], k[7]);
  cas(k[1], k[2]); cas(k[5], k[6]);
  cas(k[0], k[4]); cas(k[1], k[5]); cas(k[2], k[6]); cas(k[3], k[7]);
  cas(k[2], k[4]); cas(k[3], k[5]);
  cas(k[1], k[2]); cas(k[3], k[4]); cas(k[5], k[6]);
}

// Smallest power of two >= max(n, lo).
__device__ __forceinline__ int pow2_at_least(int n, int lo) {
  int p = lo;
  while (p < n) p <<= 1;
  return p;
}

// LDS position of key e of a sort buffer: one spare key after every eight, so
// that the threads' runs of K = 4 keys (32 bytes apart) fall on different
// banks instead of the same few (at most 2-way conflicts for 64-bit accesses).
__device__ __forceinline__ int sp(int e) { return e + (e >> 3); }

// Keys a sort buffer of n keys holds with the spare ones.
constexpr int sort_buf_keys(int n) { return n + n / 8; }

// KEYS_OUT: write the sorted keys back to keys_out instead of their ids.
// PAD_IN: `keys` is a sort buffer in LDS (positions by sp), else plain memory.
template <int NT, int K, bool KEYS_OUT = false, bool PAD_IN = false>
__device__ void merge_sort_tile(const unsigned long long* keys, uint32_t* ids, int n,
                                unsigned long long* buf0, unsigned long long* buf1,
                                unsigned long long* keys_out = nullptr) {
  const int N = pow2_at_least(n, K);
  const int t = threadIdx.x;
  const bool act = K * t < N;
  if (act) {
    unsigned long long k[K];
#pragma unroll
    for (int s = 0; s < K; ++s) {
      const int e = K * t + s;
      k[s] = e < n ? keys[PAD_IN ? sp(e) : e] : kKeyPad;
    }
    sort_network(k);
#pragma unroll
    for (int s = 0; s < K; ++s) buf0[sp(K * t + s)] = k[s];
  }
  __syncthreads();
  unsigned long long* src = buf0;
  unsigned long long* dst = buf1;
  for (int L = K; L < N; L <<= 1) {
    if (act) {
      const int pos = K * t;
      const int base = pos & ~(2 * L - 1);
      const int r = pos - base;
      const int a0 = base, b0 = base + L;     // the two runs being merged
      // number of A keys among the first r outputs (ties: A first)
      int lo = r > L ? r - L : 0, hi = r < L ? r : L;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (src[sp(a0 + mid)] <= src[sp(b0 + r - 1 - mid)]) lo = mid + 1;
        else hi = mid;
      }
      int i = lo, j = r - lo;
      unsigned long long x = i < L ? src[sp(a0 + i)] : kKeyPad;
      unsigned long long y = j < L ? src[sp(b0 + j)] : kKeyPad;
      // an exhausted run reads as all-ones keys, so one compare decides: past
      // the end of B, x <= y holds; past the end of A, it holds only if y is
      // padding too, and then either choice writes the same all-ones key
#pragma unroll
      for (int s = 0; s < K; ++s) {
        const bool take_a = x <= y;
        dst[sp(pos + s)] = take_a ? x : y;
        if (take_a) {
          ++i;
          x = i < L ? src[sp(a0 + i)] : kKeyPad;
        } else {
          ++j;
          y = j < L ? src[sp(b0 + j)] : kKeyPad;
        }
      }
    }
    __syncthreads();
    unsigned long long* tmp = src;
    src = dst;
    dst = tmp;
  }
  for (int i = t; i < n; i += NT) {
    if (KEYS_OUT)
      keys_out[i] = src[sp(i)];
    else
      ids[i] = (uint32_t)src[sp(i)];
  }
}

// The ids of the merge of two sorted key runs A[0..na) and B[0..nb) (global
// memory), each thread writing a contiguous share of the outputs after a
// merge-path search for its start (ties: A first).
__device__ void merge_runs_to_ids(const unsigned long long* A, int na,
                                  const unsigned long long* Bv, int nb, uint32_t* ids) {
  const int n = na + nb;
  const int per = (n + (int)blockDim.x - 1) / (int)blockDim.x;
  const int r = min((int)threadIdx.x * per, n), r1 = min(r + per, n);
  if (r >= r1) return;
  int lo = max(0, r - nb), hi = min(r, na);       // A keys among the first r outputs
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (A[mid] <= Bv[r - 1 - mid]) lo = mid + 1;
    else hi = mid;
  }
  int i = lo, j = r - lo;
  for (int o = r; o < r1; ++o) {
    const bool take_a = j >= nb || (i < na && A[i] <= Bv[j]);
    ids[o] = (uint32_t)(take_a ? A[i++] : Bv[j++]);
  }
}

// The tile's list is the concatenation of its run in every chunk of its
// session (chunk-major keys, run offsets in the chunks' histogram rows).
// First each run's source and place in the list (a thread per chunk, a block
// scan of the run lengths, both kept in LDS for up to kGatherChunks chunks);
// then the n keys dealt evenly over the threads, each finding the run of its
// first key by binary search and issuing its loads together.  Sessions with
// more chunks copy run by run.
constexpr int kGatherChunks = 1020;    // s_at and s_src fit in one sort buffer

template <bool PAD>
__device__ void gather_tile(const WsPtrs& W, const SessionDev& S, int lt, int n,
                            unsigned long long* dst, uint32_t* s_part, uint32_t* s_at,
                            uint32_t* s_src) {
  const int ts = S.tiles_x * S.tiles_y;
  const int nc = (S.n + kChunk - 1) / kChunk;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const bool spread = nc <= kGatherChunks;
  uint32_t carry = 0;
  for (int c0 = 0; c0 < nc; c0 += kBlock) {
    const int c = c0 + (int)threadIdx.x;
    uint32_t cnt = 0, src = 0;
    if (c < nc) {
      const uint32_t* row = W.hist + S.hist_base + (int64_t)c * ts;
      const uint32_t off = row[lt];
      const uint32_t nxt = lt + 1 < ts ? row[lt + 1] : W.chunk_total[S.chunk_base + c];
      cnt = nxt - off;
      src = W.chunk_off[S.chunk_base + c] + off;
    }
    uint32_t x = cnt;
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    if (lane == 63) s_part[wave] = x;
    __syncthreads();
    uint32_t at = carry + x - cnt, tot = 0;
    for (int q = 0; q < kBlock / 64; ++q) {
      at += q < wave ? s_part[q] : 0u;
      tot += s_part[q];
    }
    if (spread) {
      if (c < nc) {
        s_at[c] = at;
        s_src[c] = src;
      }
    } else {
      for (uint32_t j = 0; j < cnt; ++j) dst[PAD ? sp(at + j) : at + j] = W.keys[src + j];
    }
    carry += tot;
    __syncthreads();                        // s_part is reused
  }
  if (!spread) return;
  if (threadIdx.x == 0) s_at[nc] = (uint32_t)n;
  __syncthreads();
  const int per = (n + kBlock - 1) / kBlock;
  const int p0 = min((int)threadIdx.x * per, n), p1 = min(p0 + per, n);
  if (p0 >= p1) return;
  int lo = 0, hi = nc - 1;                  // last run with s_at <= p0
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (s_at[mid] <= (uint32_t)p0) lo = mid; else hi = mid - 1;
  }
  int c = lo;
  for (int q0 = p0; q0 < p1; q0 += 4) {
    unsigned long long k[4];
    int qn = min(4, p1 - q0);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (j < qn) {
        const uint32_t p = (uint32_t)(q0 + j);
        while (p >= s_at[c + 1]) ++c;       // runs are contiguous in the list
        k[j] = W.keys[s_src[c] + (p - s_at[c])];
      }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (j < qn) dst[PAD ? sp(q0 + j) : q0 + j] = k[j];
  }
}

// One workgroup per tile (neighbouring tiles on one XCD, whose L2 then holds
// the chunk rows and runs they share): lists of up to 1024 keys are gathered
// to LDS and sorted here; longer ones are gathered to the tile-major buffer
// and queued for k_sort_big_tiles.
template <bool ONE>
__global__ __launch_bounds__(kBlock) void k_sort_tiles(Batch B, WsPtrs W) {
  __shared__ unsigned long long b0[sort_buf_keys(kSortPerThread * kBlock)];
  __shared__ unsigned long long b1[sort_buf_keys(kSortPerThread * kBlock)];
  __shared__ uint32_t s_part[kBlock / 64];
  // the gather's run table lives in b0, which the merge sort fills only after
  // it has read the gathered keys from b1
  static_assert(2 * kGatherChunks + 1 <= 2 * kSortPerThread * kBlock, "run table fits b0");
  uint32_t* s_at = reinterpret_cast<uint32_t*>(b0);
  uint32_t* s_src = s_at + kGatherChunks + 1;
  const int per = (B.t_total + 7) >> 3;
  const int t = ((int)blockIdx.x & 7) * per + ((int)blockIdx.x >> 3);
  if (t >= B.t_total) return;
  const uint32_t st = W.tile_start[t];
  const int n = (int)(W.tile_start[t + 1] - st);   // all empty after an overflow
  if (n <= 0) return;
  const int s = ONE ? 0 : find_session(session_table(B), B.n_sessions, t,
                                         [](const SessionDev& x) { return x.tile_base; });
  const SessionDev& S = batch_session<ONE>(B, s);
  if (n > kSortPerThread * kBlock) {
    gather_tile<false>(W, S, t - S.tile_base, n, W.keys_tm + st, s_part, s_at, s_src);
    if (threadIdx.x == 0) {
      const unsigned long long q = atomicAdd((unsigned long long*)&W.counters[2], 1ull);
      W.big_tiles[q] = (uint32_t)t;
    }
    return;
  }
  gather_tile<true>(W, S, t - S.tile_base, n, b1, s_part, s_at, s_src);
  __syncthreads();
  merge_sort_tile<kBlock, kSortPerThread, false, true>(b1, W.ids + st, n, b0, b1);
}

// Queued long lists (gathered to the tile-major buffer): up to 4096 keys by
// the LDS merge sort with 1024 threads; up to 8192 as two such sorts of
// halves written back as keys, then one merge of the halves from global
// memory; longer ones by the bitonic network in place in global memory.  One
// launch whatever the lengths.
constexpr int kBigThreads = 1024;
constexpr int kBigKeys = kSortPerThread * kBigThreads;
__global__ __launch_bounds__(kBigThreads) void k_sort_big_tiles(WsPtrs W) {
  __shared__ unsigned long long b0[sort_buf_keys(kBigKeys)], b1[sort_buf_keys(kBigKeys)];
  const long long count = W.counters[2];
  for (long long q = blockIdx.x; q < count; q += gridDim.x) {
    const int t = (int)W.big_tiles[q];
    const int64_t st = W.tile_start[t];
    const int n = (int)(W.tile_start[t + 1] - st);
    unsigned long long* g = W.keys_tm + st;
    if (n <= kBigKeys) {
      merge_sort_tile<kBigThreads, kSortPerThread>(g, W.ids + st, n, b0, b1);
    } else if (n <= 2 * kBigKeys) {
      merge_sort_tile<kBigThreads, kSortPerThread, true>(g, nullptr, kBigKeys, b0, b1, g);
      __syncthreads();
      merge_sort_tile<kBigThreads, kSortPerThread, true>(g + kBigKeys, nullptr, n - kBigKeys, b0,
                                                          b1, g + kBigKeys);
      __threadfence_block();
      __syncthreads();
      merge_runs_to_ids(g, kBigKeys, g + kBigKeys, n - kBigKeys, W.ids + st);
    } else {
      bitonic_sort(g, n);
      for (int i = threadIdx.x; i < n; i += blockDim.x) W.ids[st + i] = (uint32_t)g[i];
    }
    __syncthreads();
  }
}

__global__ void k_debug_stage(Batch B, WsPtrs W, float* stage, int* rect, int* ranges, int* ids,
                              int64_t ids_cap) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < B.n_total) {
    if (stage) {
      const GaussRec R = W.rec[i];
      const float4 r0 = R.pos, r1 = R.conic, r2 = R.col, e = R.ext;
      float* o = stage + 12 * (int64_t)i;
      o[0] = r0.x; o[1] = r0.y; o[2] = r1.x; o[3] = r1.y; o[4] = r1.z; o[5] = r1.w;
      o[6] = r2.w; o[7] = e.x; o[8] = e.y; o[9] = r2.x; o[10] = r2.y; o[11] = r2.z;
    }
    if (rect) {
      const int4 r = W.rect[i];
      rect[4 * i + 0] = r.x; rect[4 * i + 1] = r.y; rect[4 * i + 2] = r.z; rect[4 * i + 3] = r.w;
    }
  }
  if (i < B.t_total && ranges) {
    ranges[2 * i] = (int)W.tile_start[i];
    ranges[2 * i + 1] = (int)W.tile_start[i + 1];
  }
  if (ids) {
    const int64_t total = min((int64_t)W.tile_start[B.t_total], min(W.cap, ids_cap));
    for (int64_t k = i; k < total; k += (int64_t)gridDim.x * blockDim.x) ids[k] = (int)W.ids[k];
  }
}

__global__ void k_wave_sum_test(const float* in, float* out, int n_waves) {
  constexpr int NV = kWaveSumValues;
  const int w = blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
  if (w >= n_waves) return;     // whole waves exit together
  const int lane = threadIdx.x & 63;
  float v[NV], x[3];
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = in[((int64_t)w * NV + i) * 64 + lane];
  wave_reduce_scatter<NV>(v, x);
  if ((lane & 15) == 15) {
    const int row = lane >> 4;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const int idx = wave_scatter_index(NV, row, j);
      if (idx >= 0) out[(int64_t)w * NV + idx] = x[j];
    }
  }
}

}  // namespace

hipError_t launch_forward_prep(const Batch& b, const WsPtrs& w, unsigned long long* max_pairs,
                               bool reuse_lists, hipStream_t st, StageTimer* tm) {
  const bool one = b.n_sessions == 1;
  if (reuse_lists) {
    if (b.b_total > 0) {
      Scope sc(tm, kStPreprocess, st);
      if (one)
        k_preprocess<true, true><<<b.b_total, kGaussPerBlock, 0, st>>>(b, w);
      else
        k_preprocess<true, false><<<b.b_total, kGaussPerBlock, 0, st>>>(b, w);
    }
    return hipGetLastError();
  }
  const size_t lds = sizeof(uint32_t) * (size_t)(b.t_max > 0 ? b.t_max : 1);
  if (b.b_total <= 0) {
    // no Gaussians: k_preprocess (which zeroes the counters) does not run
    Scope sc(tm, kStInit, st);
    k_init<<<1, 64, 0, st>>>(w.counters);
  }
  if (b.b_total > 0) {
    Scope sc(tm, kStPreprocess, st);
    if (one)
      k_preprocess<false, true><<<b.b_total, kGaussPerBlock, 0, st>>>(b, w);
    else
      k_preprocess<false, false><<<b.b_total, kGaussPerBlock, 0, st>>>(b, w);
  }
  if (b.c_total > 0) {
    Scope sc(tm, kStBinCount, st);
    if (one)
      k_chunk_hist<true><<<b.c_total, kBinThreads, lds, st>>>(b, w);
    else
      k_chunk_hist<false><<<b.c_total, kBinThreads, lds, st>>>(b, w);
  }
  {
    Scope sc(tm, kStScan, st);
    const dim3 grid((b.t_total + kBlock - 1) / kBlock, kScanGroups);
    if (one)
      k_tile_group_sums<true><<<grid, kBlock, 0, st>>>(b, w);
    else
      k_tile_group_sums<false><<<grid, kBlock, 0, st>>>(b, w);
    k_scan_tiles<<<1, kScanThreads, 0, st>>>(w, b.t_total, b.c_total, max_pairs);
  }
  if (b.c_total > 0) {
    Scope sc(tm, kStEmit, st);
    const size_t lds_emit = lds + sizeof(uint16_t) * kStagePairs;
    if (one)
      k_emit<true><<<b.c_total, kBinThreads, lds_emit, st>>>(b, w);
    else
      k_emit<false><<<b.c_total, kBinThreads, lds_emit, st>>>(b, w);
  }
  if (b.t_total > 0) {
    Scope sc(tm, kStSort, st);
    if (one)
      k_sort_tiles<true><<<8 * ((b.t_total + 7) / 8), kBlock, 0, st>>>(b, w);
    else
      k_sort_tiles<false><<<8 * ((b.t_total + 7) / 8), kBlock, 0, st>>>(b, w);
    k_sort_big_tiles<<<b.t_total < 512 ? b.t_total : 512, kBigThreads, 0, st>>>(w);
  }
  return hipGetLastError();
}

hipError_t launch_debug_stage(const Batch& b, const WsPtrs& w, float* stage, int* rect,
                              int* ranges, int* ids, int64_t ids_cap, hipStream_t st) {
  const int n = b.n_total > b.t_total ? b.n_total : b.t_total;
  const int grid = (n + 255) / 256 > 0 ? (n + 255) / 256 : 1;
  k_debug_stage<<<grid, 256, 0, st>>>(b, w, stage, rect, ranges, ids, ids_cap);
  return hipGetLastError();
}

hipError_t launch_wave_sum_test(const float* in, float* out, int n_waves, hipStream_t st) {
  if (n_waves <= 0) return hipSuccess;
  k_wave_sum_test<<<(n_waves + 3) / 4, 256, 0, st>>>(in, out, n_waves);
  return hipGetLastError();
}

}  // namespace rtgs
