// Step 3 (rendering: alpha computing, Eq. 2, and alpha blending, Eq. 3) and
// Step 4 (rendering backpropagation, the exact derivative of Eq. 3 that
// Eqs. 4-5 sketch) for a batch of sessions sharing one tile space.
//
// One workgroup per 16x16 tile, 256 lanes = 4 wave64; each wave owns an 8x8
// quadrant, so a Gaussian whose padded bounding box misses a quadrant is
// skipped by that whole wave (a wave-uniform branch; the GPU counterpart of
// the paper's 4x4 subtiles).  Gaussian records of the tile's depth-sorted
// list are staged through LDS in batches of 256.
//
// Forward: per lane, alpha = min(0.99, o exp(power)); skip alpha < 1/255;
// stop before T would fall below 1e-4; saves final T and the position of the
// last blended pair (the per-pixel state the backward reuses instead of
// re-running the forward, the role of the paper's R&B buffer, Sec. 5.2).
// With a session's loss targets it also writes the gradient of the L1 loss
// (Eq. 6) of every pixel it writes, so no loss pass reads the image back.
//
// Backward: walks the list from the block's largest saved position down,
// recovering T before each blended fragment as T / (1 - alpha) (Eq. 5 read
// as the reverse recurrence) and the normalised suffix colour/depth; the
// per-fragment 2D gradients of one list entry are summed over the wave by a
// reduce-scatter (lane swaps across halves and rows, then DPP row sums), the
// four waves' sums are added in LDS in a fixed order, and the tile's total for
// that Gaussian is stored in the pair's own slot: the pixel -> tile merge of
// the paper's Gradient Merging Unit (Sec. 5.3) done with cross-lane
// operations.  The tile -> Gaussian merge (its Stage Buffer) is a segmented
// sum over the Gaussian's slots in the preprocessing backward; no float
// atomics anywhere, so gradients are bitwise reproducible.
#include "rtgs_internal.h"

namespace rtgs {
namespace {

__device__ __forceinline__ int tile_of_block(int t_total) {
  // Workgroups are dealt round-robin to the 8 XCDs; give each XCD a contiguous
  // band of tiles so neighbouring tiles share its L2.
  const int per = (t_total + 7) >> 3;
  return ((int)blockIdx.x & 7) * per + ((int)blockIdx.x >> 3);
}

// A tile holds 16x16 samples: one per pixel normally, or one per block of
// 2^sub_sx x 2^sub_sy pixels for a downsampled frame (the pixel the mask keeps
// in that block).  Wave w owns the 8x8 samples of quadrant w.
struct TileCtx {
  int s;
  int lt;                       // tile index within the session
  int tile_x0, tile_y0;         // first pixel of the tile
  int bx0, by0;                 // first pixel of this lane's sample block
  int px, py;                   // the lane's sample pixel
  bool inside;                  // the block lies (partly) in the image
  bool has;                     // a sample pixel exists (mask) in the block
  int pix;
  unsigned wbit;
};

// The sample a thread takes by default: wave w the 8x8 quadrant w.
__device__ __forceinline__ int quadrant_sample() {
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  return ((wave >> 1) * 8 + (lane >> 3)) * 16 + (wave & 1) * 8 + (lane & 7);
}

// sidx: the thread's sample of the tile, row-major 0..255.
template <bool ONE>
__device__ __forceinline__ TileCtx tile_ctx(const Batch& B, int tile, int sidx) {
  TileCtx c;
  c.s = ONE ? 0
            : find_session(session_table(B), B.n_sessions, tile,
                           [](const SessionDev& x) { return x.tile_base; });
  const SessionDev& S = batch_session<ONE>(B, c.s);
  c.lt = tile - S.tile_base;
  c.tile_x0 = (c.lt % S.tiles_x) << (4 + S.sub_sx);
  c.tile_y0 = (c.lt / S.tiles_x) << (4 + S.sub_sy);
  const int wave = (int)threadIdx.x >> 6;
  const int sx = sidx & 15, sy = sidx >> 4;
  c.bx0 = c.tile_x0 + (sx << S.sub_sx);
  c.by0 = c.tile_y0 + (sy << S.sub_sy);
  c.inside = c.bx0 < S.width && c.by0 < S.height;
  c.px = c.bx0;
  c.py = c.by0;
  c.has = c.inside;
  if (c.inside && (S.sub_sx | S.sub_sy)) {
    // the block's sample: its first masked-in pixel in raster order
    c.has = false;
    const int x1 = min(S.width, c.bx0 + (1 << S.sub_sx));
    const int y1 = min(S.height, c.by0 + (1 << S.sub_sy));
    for (int y = c.by0; y < y1 && !c.has; ++y)
      for (int x = c.bx0; x < x1; ++x)
        if (S.pmask[y * S.width + x]) {
          c.px = x;
          c.py = y;
          c.has = true;
          break;
        }
  }
  c.pix = c.py * S.width + c.px;
  c.wbit = 1u << wave;
  return c;
}

// Smallest value of the quadratic form q(d) = a dx^2 + 2 b dx dy + c dy^2
// over the box [x0, x1] x [y0, y1] of offsets d (a convex quadratic: zero if
// the box holds the centre, otherwise reached on an edge, where it is a 1D
// quadratic minimised in closed form and clamped to the edge).
// ia, ic: 1/a and 1/c (0 where a or c is not positive), shared by the four
// quadrants of an entry.
__device__ __forceinline__ float box_min_quad(float a, float b, float c, float ia, float ic,
                                              float x0, float x1, float y0, float y1) {
  if (x0 <= 0.f && x1 >= 0.f && y0 <= 0.f && y1 >= 0.f) return 0.f;
  float m = 3.0e38f;
  const float xs[2] = {x0, x1}, ys[2] = {y0, y1};
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    const float X = xs[e];                           // edge dx = X
    const float dy = fminf(y1, fmaxf(y0, -b * X * ic));
    m = fminf(m, a * X * X + 2.f * b * X * dy + c * dy * dy);
    const float Y = ys[e];                           // edge dy = Y
    const float dx = fminf(x1, fmaxf(x0, -b * Y * ia));
    m = fminf(m, a * dx * dx + 2.f * b * dx * Y + c * Y * Y);
  }
  return m;
}

// Bit w set when the alpha >= 1/255 ellipse (q <= t) of the Gaussian can
// reach a pixel centre of the quadrant of wave w (8x8 sample blocks of
// 2^sx x 2^sy pixels).  The margin keeps the test conservative against the
// float32 evaluation of alpha.
__device__ __forceinline__ unsigned quad_mask(float4 r0, float4 r1, float4 ex, int tx0, int ty0,
                                              int sx, int sy) {
  const float u = r0.x + r0.z, v = r0.y + r0.w;
  const float t = ex.z * (1.f + 1e-3f) + 1e-3f;
  const float wx = (float)((8 << sx) - 1), wy = (float)((8 << sy) - 1);
  const float ia = r1.x > 0.f ? 1.f / r1.x : 0.f, ic = r1.z > 0.f ? 1.f / r1.z : 0.f;
  unsigned m = 0;
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    const float qx = (float)(tx0 + ((w & 1) * 8 << sx)) + 0.5f - u;
    const float qy = (float)(ty0 + ((w >> 1) * 8 << sy)) + 0.5f - v;
    const float q = box_min_quad(r1.x, r1.y, r1.z, ia, ic, qx, qx + wx, qy, qy + wy);
    m |= (q <= t) ? (1u << w) : 0u;
  }
  return m;
}

// The same test against four boxes of samples, (x0, y0, x1, y1) inclusive,
// one per wave (the lanes of a wave assigned by previous work).
__device__ __forceinline__ unsigned box_mask(float4 r0, float4 r1, float4 ex, int tx0, int ty0,
                                             int sx, int sy, const int4* boxes) {
  const float u = r0.x + r0.z, v = r0.y + r0.w;
  const float t = ex.z * (1.f + 1e-3f) + 1e-3f;
  const float ia = r1.x > 0.f ? 1.f / r1.x : 0.f, ic = r1.z > 0.f ? 1.f / r1.z : 0.f;
  unsigned m = 0;
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    const int4 bx = boxes[w];
    const float qx0 = (float)(tx0 + (bx.x << sx)) + 0.5f - u;
    const float qy0 = (float)(ty0 + (bx.y << sy)) + 0.5f - v;
    const float qx1 = (float)(tx0 + ((bx.z + 1) << sx) - 1) + 0.5f - u;
    const float qy1 = (float)(ty0 + ((bx.w + 1) << sy) - 1) + 0.5f - v;
    const float q = box_min_quad(r1.x, r1.y, r1.z, ia, ic, qx0, qx1, qy0, qy1);
    m |= (q <= t) ? (1u << w) : 0u;
  }
  return m;
}

// 64-bit ballot of "entry (base + lane) is in this wave's quadrant".
__device__ __forceinline__ unsigned long long wave_entries(const unsigned* s_m, int base, int cnt,
                                                           unsigned wbit) {
  const int k = base + (int)(threadIdx.x & 63);
  const bool hit = k < cnt && (s_m[k] & wbit) != 0;
  return __ballot(hit);
}

// Saved fragments (the per-fragment state of the paper's R&B buffer): for
// every list entry a wave evaluates, the 64-bit mask of its lanes that
// blended it, and for those lanes, in entry order and compacted by lane rank,
// (alpha, 1 - alpha) with alpha negated where it was clamped to 0.99.  The
// stream of wave w of a tile with list [start, end) begins at float2 index
// 64 (4 start + w (end - start)): room for every lane blending every entry.
__device__ __forceinline__ int64_t frag_base(int start, int end, int wave) {
  return 64 * (4 * (int64_t)start + (int64_t)wave * (end - start));
}

__device__ __forceinline__ uint32_t lane_rank(unsigned long long m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Lanes assigned by previous work (the GPU form of the paper's workload
// scheduling unit, Sec. 5.2): the tile's 256 samples sorted by the list
// entries each walked in a previous forward (S.lane_work; ties and missing
// values by sample index), wave w taking ranks 64 w to 64 w + 63, so each
// wave's lanes finish together.  Each wave culls against the bounding box of
// its samples.  Writes the permutation for the backward and the boxes to LDS.
__device__ __forceinline__ int lane_schedule(const SessionDev& S, const WsPtrs& W, int tile,
                                             int tile_x0, int tile_y0, uint32_t* s_key,
                                             uint8_t* s_pix, int4* s_box) {
  const int tid = threadIdx.x;
  const int bx = tile_x0 + ((tid & 15) << S.sub_sx), by = tile_y0 + ((tid >> 4) << S.sub_sy);
  uint32_t work = 0;
  if (S.lane_work && bx < S.width && by < S.height) work = S.lane_work[by * S.width + bx];
  const uint32_t key = (work << 8) | (uint32_t)tid;
  s_key[tid] = key;
  __syncthreads();
  int rank = 0;
  for (int j = 0; j < kBlock; ++j) rank += s_key[j] < key ? 1 : 0;
  s_pix[rank] = (uint8_t)tid;
  __syncthreads();
  const int sidx = s_pix[tid];
  W.lane_perm[(int64_t)tile * kBlock + tid] = (uint8_t)sidx;
  int x0 = sidx & 15, x1 = x0, y0 = sidx >> 4, y1 = y0;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    x0 = min(x0, __shfl_xor(x0, off));
    x1 = max(x1, __shfl_xor(x1, off));
    y0 = min(y0, __shfl_xor(y0, off));
    y1 = max(y1, __shfl_xor(y1, off));
  }
  if ((tid & 63) == 0) s_box[tid >> 6] = make_int4(x0, y0, x1, y1);
  __syncthreads();
  return sidx;
}

// STATS: also count, per pixel, the fragments blended and the list entries
// visited (the work counts of a frame); off in ordinary renders.
// FRAG: also save the fragments' alpha (see frag_base).
// BAL: lanes assigned by previous work (lane_schedule); also writes each
// sample's walked entries to S.lane_work_out for the next forward.
template <bool STATS, bool FRAG, bool BAL, bool ONE>
__global__ __launch_bounds__(kBlock) void k_raster_fwd(Batch B, WsPtrs W) {
  __shared__ float4 s_r0[kBlock], s_r1[kBlock], s_r2[kBlock];
  __shared__ unsigned s_m[kBlock];
  __shared__ uint32_t s_key[BAL ? kBlock : 1];
  __shared__ uint8_t s_pix[BAL ? kBlock : 1];
  __shared__ int4 s_box[4];
  const int tile = tile_of_block(B.t_total);
  if (tile >= B.t_total) return;
  int sidx = quadrant_sample();
  if (BAL) {
    const TileCtx c0 = tile_ctx<ONE>(B, tile, sidx);
    sidx = lane_schedule(batch_session<ONE>(B, c0.s), W, tile, c0.tile_x0, c0.tile_y0, s_key,
                         s_pix, s_box);
  }
  const TileCtx c = tile_ctx<ONE>(B, tile, sidx);
  const SessionDev& S = batch_session<ONE>(B, c.s);
  const int tid = threadIdx.x;
  const bool active = c.has && (S.pmask == nullptr || S.pmask[c.pix] != 0);
  const float pxf = (float)c.px + 0.5f, pyf = (float)c.py + 0.5f;
  // list positions fit in int32: the pair capacity is below 2^31
  const int start = (int)min((int64_t)W.tile_start[tile], W.cap);
  const int end = (int)min((int64_t)W.tile_start[tile + 1], W.cap);
  // T carries the pixel's stop in its sign: T > 0 while the pixel walks
  // (T >= 1e-4 > 0 until the stop), -T once it has stopped (or never walks),
  // so the per-entry test is one compare and no flag is carried across the loop
  float T = active ? 1.f : -1.f, C0 = 0.f, C1 = 0.f, C2 = 0.f, D = 0.f;
  int last = -1;
  int stop = end;               // list position where the pixel stopped
  int nblend = 0;
  const int fwave = tid >> 6, flane = tid & 63;
  uint32_t fcur = 0;            // saved fragments of this wave so far
  const int64_t fbase = FRAG ? frag_base(start, end, fwave) : 0;
  // the Gaussian id this thread stages next (loaded one batch ahead)
  uint32_t nid = start + tid < end ? W.ids[start + tid] : 0u;
  for (int b0 = start; b0 < end; b0 += kBlock) {
    if (__syncthreads_and(!(T > 0.f))) break;
    const int e = b0 + tid;
    if (e < end) {
      const GaussRec r = W.rec[nid];
      s_r0[tid] = r.pos;
      s_r1[tid] = conic_log2(r.conic);
      s_r2[tid] = r.col;
      const unsigned qm = BAL ? box_mask(r.pos, r.conic, r.ext, c.tile_x0, c.tile_y0, S.sub_sx,
                                         S.sub_sy, s_box)
                              : quad_mask(r.pos, r.conic, r.ext, c.tile_x0, c.tile_y0, S.sub_sx,
                                          S.sub_sy);
      s_m[tid] = qm;
      W.qmask[e] = (uint8_t)qm;     // for the backward, which walks no entry unstaged here
    }
    if (e + kBlock < end) nid = W.ids[e + kBlock];
    __syncthreads();
    const int cnt = min(kBlock, end - b0);
    // the lane's last blended entry of this batch, as its LDS byte offset
    // (16 k, the address the step reads anyway)
    int last16 = -1;
    for (int q = 0; q < kBlock / 64; ++q) {
      unsigned long long m = wave_entries(s_m, 64 * q, cnt, c.wbit);
      // every lane evaluates each entry; the decisions are selects, not
      // branches: skip (alpha < 1/255), stop (T would fall below 1e-4; the
      // fragment is excluded) or blend
      auto step = [&](int k) {
        const Frag f = frag_alpha(s_r0[k], s_r1[k], pxf, pyf);
        const float tn = T * f.om;
        const bool hit = T > 0.f && !(f.alpha < kAlphaMin);
        const bool blend = hit && !(tn < kTMin);
        const bool stop_here = hit != blend;              // hit and T would fall below 1e-4
        if (STATS || BAL) stop = stop_here ? b0 + k : stop;
        const float w = blend ? f.alpha * T : 0.f;       // adds exactly 0 otherwise
        const float4 col = s_r2[k];
        C0 = __builtin_fmaf(w, col.x, C0);
        C1 = __builtin_fmaf(w, col.y, C1);
        C2 = __builtin_fmaf(w, col.z, C2);
        D = __builtin_fmaf(w, col.w, D);
        T = blend ? tn : (stop_here ? -T : T);
        last16 = blend ? (k << 4) : last16;
        if (STATS) nblend += blend ? 1 : 0;
        if (FRAG) {
          const unsigned long long bm = __ballot(blend);
          if (flane == 0) W.fmask[(int64_t)(b0 + k) * 4 + fwave] = bm;
          if (blend) {
            const float4 k4 = s_r1[k];
            W.fdata[fbase + fcur + lane_rank(bm)] =
                make_float2(k4.w * f.e > kAlphaMax ? -f.alpha : f.alpha, f.om);
          }
          fcur += (uint32_t)__popcll(bm);
        }
      };
      while (m) {
        if (__ballot(T > 0.f) == 0) break;             // the whole wave has stopped
        step(64 * q + __builtin_ctzll(m));
        m &= m - 1;
        if (m) {                                       // two entries per check
          step(64 * q + __builtin_ctzll(m));
          m &= m - 1;
        }
      }
    }
    last = last16 >= 0 ? b0 + (last16 >> 4) : last;
    __syncthreads();
  }
  if (FRAG && flane == 0) W.fcount[(int64_t)tile * 4 + fwave] = fcur;
  T = fabsf(T);
  if (!c.inside) return;
  if (BAL && S.lane_work_out) {
    const int walked = active ? min(stop + 1, end) - start : 0;
    S.lane_work_out[c.by0 * S.width + c.bx0] = (uint16_t)min(walked, 65535);
  }
  const int64_t hw = (int64_t)S.width * S.height;
  // loss gradient (Eq. 6, L1 colour and depth, means over the active pixels):
  // the arithmetic of the separate loss pass on the values written here
  float l1_sc = 0.f, l1_sd = 0.f;
  if (S.l1_dcolor) {
    const float n = S.l1_n_active ? fmaxf((float)*S.l1_n_active, 1.f) : (float)hw;
    l1_sc = S.l1_w_color / (3.f * n);
    l1_sd = S.l1_w_depth / n;
  }
  // every pixel of the lane's block: the sample gets its result, the others
  // (masked out) render as background
  const int x1 = min(S.width, c.bx0 + (1 << S.sub_sx));
  const int y1 = min(S.height, c.by0 + (1 << S.sub_sy));
  for (int y = c.by0; y < y1; ++y)
    for (int x = c.bx0; x < x1; ++x) {
      const int p = y * S.width + x;
      const bool me = p == c.pix;
      if (S.color) {
        S.color[p] = me ? C0 : 0.f;
        S.color[hw + p] = me ? C1 : 0.f;
        S.color[2 * hw + p] = me ? C2 : 0.f;
      }
      if (S.l1_dcolor) {
        const float m = S.pmask ? (S.pmask[p] ? 1.f : 0.f) : 1.f;
        const float v[4] = {me ? C0 : 0.f, me ? C1 : 0.f, me ? C2 : 0.f, me ? D : 0.f};
#pragma unroll
        for (int k = 0; k < 3; ++k)
          S.l1_dcolor[k * hw + p] = m * l1_sc * sign_of(v[k] - S.l1_tcolor[k * hw + p]);
        S.l1_ddepth[p] = m * l1_sd * sign_of(v[3] - S.l1_tdepth[p]);
      }
      if (S.depth) S.depth[p] = me ? D : 0.f;
      if (S.alpha) S.alpha[p] = me ? 1.f - T : 0.f;
      if (S.final_T) S.final_T[p] = me ? T : 1.f;
      if (S.last_idx) S.last_idx[p] = me ? last : -1;
      if (STATS && S.stats) {
        // work counts: fragments blended, list entries up to the stop (or
        // the end of the list), list entries up to the last blended one
        S.stats[p] = me ? nblend : 0;
        S.stats[hw + p] = me && active ? min(stop + 1, end) - start : 0;
        S.stats[2 * hw + p] = me && last >= 0 ? last - start + 1 : 0;
      }
    }
}

constexpr int kBwdBatch = 64;            // list entries staged per batch

// Gaussian-major slot of the pair (Gaussian g, tile (tx, ty)): g's first slot
// plus the tile's row-major index inside g's tile rectangle.
__device__ __forceinline__ int64_t pair_slot(const WsPtrs& W, uint32_t g, int tx, int ty) {
  const int4 r = W.rect[g];
  return (int64_t)W.goff[g] + (ty - r.y) * (r.z - r.x + 1) + (tx - r.x);
}

// NV = 10 (all parameters: u, v, a, b, c, o, r, g, b, z) or 6 (pose only:
// u, v, a, b, c, z).  GA: some session has an alpha-image gradient (without
// one, its term of dL/dalpha is left out rather than added as zero).  Each
// (tile, Gaussian) pair gets the sum of its pixels' gradients in slot
// pair_slot(); the sum is formed in a fixed order (lane swaps and DPP row sums
// inside each wave, then the four waves in order), so the result is bitwise
// reproducible and no float atomics are used.  Eight waves per SIMD: the
// compiler is held to 64 VGPRs.
// FRAG: the forward saved its fragments (frag_base): each entry's blending
// lanes and their (alpha, 1 - alpha) are read instead of re-evaluating alpha,
// and entries no lane of the wave blended are skipped without arithmetic; the
// values are those the forward computed, so the gradients are bitwise those
// of the re-evaluating form.
// BAL: the forward assigned lanes by previous work (lane_schedule); the same
// samples go to the same lanes here (the saved quadrant bits are per wave).
template <int NV, bool GA, bool FRAG, bool BAL, bool ONE>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8)))
void k_raster_bwd(Batch B, WsPtrs W) {
  constexpr int kStride = NV + 1;          // odd stride: conflict-free epilogue reads
  __shared__ float4 s_r0[kBwdBatch], s_r1[kBwdBatch], s_r2[kBwdBatch], s_cn[kBwdBatch];
  __shared__ unsigned s_m[kBwdBatch];
  __shared__ unsigned long long s_fm[FRAG ? 4 : 1][FRAG ? kBwdBatch : 1];
  // per wave: kStride floats per entry, then one float that takes the
  // reduce-scatter outputs no entry needs; rows padded to 16 bytes so they
  // are cleared with 16-byte stores
  constexpr int kPartRow = (kBwdBatch * kStride + 1 + 3) & ~3;
  __shared__ __align__(16) float s_part[4][kPartRow];
  __shared__ int s_hi;
  const int tile = tile_of_block(B.t_total);
  if (tile >= B.t_total) return;
  const int sidx = BAL ? (int)W.lane_perm[(int64_t)tile * kBlock + threadIdx.x] : quadrant_sample();
  const TileCtx c = tile_ctx<ONE>(B, tile, sidx);
  const SessionDev& S = batch_session<ONE>(B, c.s);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int ltx = c.lt % S.tiles_x, lty = c.lt / S.tiles_x;
  const bool active = c.has && (S.pmask == nullptr || S.pmask[c.pix] != 0);
  const int64_t hw = (int64_t)S.width * S.height;
  int last = -1;
  float Tc = 1.f, g0 = 0.f, g1 = 0.f, g2 = 0.f, gD = 0.f, gA = 0.f;
  if (active) {
    last = S.last_idx[c.pix];
    Tc = S.final_T[c.pix];
    g0 = S.dl_color[c.pix];
    g1 = S.dl_color[hw + c.pix];
    g2 = S.dl_color[2 * hw + c.pix];
    gD = S.dl_depth[c.pix];
    if (GA && S.dl_alpha) gA = S.dl_alpha[c.pix];
  }
  const float gAT = gA * Tc;        // dA/dalpha_j = T_final / (1 - alpha_j)
  if (tid == 0) s_hi = -1;
  __syncthreads();
  if (last >= 0) atomicMax(&s_hi, last);
  __syncthreads();
  const int start = (int)min((int64_t)W.tile_start[tile], W.cap);
  const int end = (int)min((int64_t)W.tile_start[tile + 1], W.cap);
  // a saved position outside this tile's list (state of another forward) is
  // never followed past the list
  const int hi = min(s_hi, end - 1);
  const float pxf = (float)c.px + 0.5f, pyf = (float)c.py + 0.5f;
  // saved fragments: this wave's last blended position, its stream and cursor
  int wave_last = last;
  uint32_t fcur = 0;
  int64_t fbase = 0;
  if (FRAG) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) wave_last = max(wave_last, __shfl_xor(wave_last, off));
    fcur = W.fcount[(int64_t)tile * 4 + wave];
    fbase = frag_base(start, end, wave);
  }
  // S_j . g: the colour and depth of the fragments behind j, normalised by
  // the transmittance T_{j+1} they start from, dotted with the upstream gradient
  float SG = 0.f;
  float* part = s_part[wave];
  // the Gaussian id this thread stages next (loaded one batch ahead)
  uint32_t nid = 0;
  {
    const int b0 = max(hi + 1 - kBwdBatch, start);
    if (tid < hi + 1 - b0) nid = W.ids[b0 + tid];
  }
  for (int bend = hi + 1; bend > start; bend -= kBwdBatch) {
    const int b0 = max(bend - kBwdBatch, start);
    const int cnt = bend - b0;
    const int lrel = last - b0;     // entries k <= lrel lie before the pixel's stop
    const uint32_t gid = nid;       // Gaussian of entry b0 + tid (tid < cnt)
    __syncthreads();
    if (tid < cnt) {
      const GaussRec r = W.rec[gid];
      s_r0[tid] = r.pos;
      s_r1[tid] = conic_log2(r.conic);
      s_r2[tid] = r.col;
      s_cn[tid] = r.conic;
      // the forward staged every entry up to the last blended one of any
      // pixel of the tile, and saved its quadrant mask
      s_m[tid] = W.qmask[b0 + tid];
      if (FRAG) {
        // blend masks; a wave reads only entries up to its last blend, all of
        // which its forward evaluated and wrote
        const ulonglong2* fm = reinterpret_cast<const ulonglong2*>(W.fmask + (int64_t)(b0 + tid) * 4);
        const ulonglong2 a = fm[0], b = fm[1];
        s_fm[0][tid] = a.x;
        s_fm[1][tid] = a.y;
        s_fm[2][tid] = b.x;
        s_fm[3][tid] = b.y;
      }
    }
    {
      const int nb0 = max(b0 - kBwdBatch, start);
      if (tid < b0 - nb0) nid = W.ids[nb0 + tid];
    }
    // zero this batch's partial sums (each wave its own)
    for (int i = lane; i < kBwdBatch * kStride / 4; i += 64)
      reinterpret_cast<float4*>(part)[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    __syncthreads();
    for (int q = kBwdBatch / 64 - 1; q >= 0; --q) {
      unsigned long long m = wave_entries(s_m, 64 * q, cnt, c.wbit);
      auto step = [&](int k) {
        const float4 k4 = s_r1[k];
        Frag f;
        bool contrib, clamped;
        if (FRAG) {
          if (b0 + k > wave_last) return;                // after every blend of the wave
          const unsigned long long bm = s_fm[wave][k];
          if (bm == 0) return;                           // no lane blended this entry
          fcur -= (uint32_t)__popcll(bm);
          contrib = ((bm >> lane) & 1ull) != 0;
          float2 rec = make_float2(0.f, 1.f);
          if (contrib) rec = W.fdata[fbase + fcur + lane_rank(bm)];
          const float4 r0 = s_r0[k];
          f.dx = (r0.x - pxf) + r0.z;
          f.dy = (r0.y - pyf) + r0.w;
          f.alpha = fabsf(rec.x);
          f.om = rec.y;
          clamped = rec.x < 0.f;
        } else {
          f = frag_alpha(s_r0[k], k4, pxf, pyf);
          contrib = k <= lrel && !(f.alpha < kAlphaMin);
          if (__ballot(contrib) == 0) return;            // no lane blended this entry
          clamped = k4.w * f.e > kAlphaMax;
        }
        // lanes that did not blend it take alpha = 0 and 1 - alpha = 1, so
        // every update below leaves their state unchanged and their
        // gradients exactly zero (selects, not branches)
        const float4 col = s_r2[k];
        const float al = contrib ? f.alpha : 0.f;
        const float om = contrib ? f.om : 1.f;
        const float rom = __builtin_amdgcn_rcpf(om);
        const float Tj = Tc * rom;                     // T before this fragment (rcp(1) = 1)
        const float w = al * Tj;
        // (colour, depth) of the fragment dotted with the upstream gradient
        float cg = col.x * g0;
        cg = __builtin_fmaf(col.y, g1, cg);
        cg = __builtin_fmaf(col.z, g2, cg);
        cg = __builtin_fmaf(col.w, gD, cg);
        // dL/dalpha_j = T_j (c_j - S_j) . g + T_final gA / (1 - alpha_j)
        const float dla = GA ? __builtin_fmaf(Tj, cg - SG, gAT * rom) : Tj * (cg - SG);
        SG = __builtin_fmaf(al, cg, om * SG);
        Tc = Tj;
        // the clamp alpha = 0.99 has no gradient to o or to the power
        const bool live = contrib && !clamped;
        const float ng = live ? -(f.alpha * dla) : 0.f;  // -dL/dpower
        const float pg = ng * f.dx, qg = ng * f.dy;
        // summed over the tile's pixels, these give the 2D gradients once
        // the Gaussian's conic is applied (epilogue)
        float v[NV];
        v[0] = pg;
        v[1] = qg;
        v[2] = pg * f.dx;
        v[3] = pg * f.dy;
        v[4] = qg * f.dy;
        v[NV - 1] = w * gD;                               // depth slot (last)
        if (NV == 10) {
          v[5] = ng;                                      // o dL/do (epilogue)
          v[6] = w * g0;
          v[7] = w * g1;
          v[8] = w * g2;
        }
        float x[3];
        wave_reduce_scatter<NV>(v, x);
        if ((lane & 15) == 15) {
          const int row = lane >> 4;
          // x[j] is value wave_scatter_index(NV, row, j): that of j = 0 plus
          // 2 j, or for the output only odd rows carry, that minus 1; even
          // rows write that output to the spare float, so every store is
          // made by all four row ends at once
          float* dst = part + k * kStride + wave_scatter_index(NV, row, 0);
#pragma unroll
          for (int j = 0; j < 3; ++j) {
            if (1 + 2 * j < NV / 2)
              dst[2 * j] = x[j];
            else if (2 * j < NV / 2)
              ((row & 1) ? dst : part + kBwdBatch * kStride + 1 - 2 * j)[2 * j - 1] = x[j];
          }
        }
      };
      while (m) {
        // descending list order, two entries per iteration (their alpha
        // evaluations are independent and can overlap)
        const int b1 = 63 - __builtin_clzll(m);
        m &= ~(1ull << b1);
        step(64 * q + b1);
        if (m) {
          const int b2 = 63 - __builtin_clzll(m);
          m &= ~(1ull << b2);
          step(64 * q + b2);
        }
      }
    }
    __syncthreads();
    if (tid < cnt) {
      const int64_t slot = pair_slot(W, gid, ltx, lty);
      if (slot < W.cap) {
        float t[NV];
#pragma unroll
        for (int i = 0; i < NV; ++i) {
          const int o = tid * kStride + i;
          t[i] = ((s_part[0][o] + s_part[1][o]) + s_part[2][o]) + s_part[3][o];
        }
        // d power / d(u, v) = -(a dx + b dy, b dx + c dy) and
        // d power / d(a, b, c) = -(dx^2 / 2, dx dy, dy^2 / 2): the sums of
        // p = -g dx and q = -g dy (g = dL/dpower) and of p dx, p dy, q dy
        // become the 2D gradients with the conic applied once here
        const float4 cn = s_cn[tid];
        float* dst = W.partial + slot * NV;
        dst[0] = __builtin_fmaf(cn.x, t[0], cn.y * t[1]);
        dst[1] = __builtin_fmaf(cn.y, t[0], cn.z * t[1]);
        dst[2] = 0.5f * t[2];
        dst[3] = t[3];
        dst[4] = 0.5f * t[4];
        // alpha = o e below the clamp, so dalpha/do = e = alpha / o and
        // dL/do = sum alpha dL/dalpha / o = -(sum of -dL/dpower) / o
        if (NV == 10) dst[5] = -t[5] / cn.w;
#pragma unroll
        for (int i = NV == 10 ? 6 : 5; i < NV; ++i) dst[i] = t[i];
      }
    }
  }
  // pairs after the last blended fragment of every pixel carry no gradient
  const int z0 = max(hi + 1, start);
  for (int pos = z0 + tid; pos < end; pos += kBlock) {
    const uint32_t g = W.ids[pos];
    const int64_t slot = pair_slot(W, g, ltx, lty);
    if (slot < W.cap) {
      float* dst = W.partial + slot * NV;
#pragma unroll
      for (int i = 0; i < NV; ++i) dst[i] = 0.f;
    }
  }
}

}  // namespace

template <bool STATS>
static void raster_fwd_variant(const Batch& b, const WsPtrs& w, bool frags, bool bal, int grid,
                               hipStream_t st) {
  if (frags) {
    if (bal)
      k_raster_fwd<STATS, true, true, false><<<grid, kBlock, 0, st>>>(b, w);
    else
      k_raster_fwd<STATS, true, false, false><<<grid, kBlock, 0, st>>>(b, w);
  } else {
    if (bal)
      k_raster_fwd<STATS, false, true, false><<<grid, kBlock, 0, st>>>(b, w);
    else if (b.n_sessions == 1)
      k_raster_fwd<STATS, false, false, true><<<grid, kBlock, 0, st>>>(b, w);
    else
      k_raster_fwd<STATS, false, false, false><<<grid, kBlock, 0, st>>>(b, w);
  }
}

hipError_t launch_raster_fwd(const Batch& b, const WsPtrs& w, bool stats, bool frags, bool bal,
                             hipStream_t st, StageTimer* tm) {
  if (b.t_total <= 0) return hipSuccess;
  const int grid = 8 * ((b.t_total + 7) / 8);
  Scope sc(tm, kStRasterFwd, st);
  if (stats)
    raster_fwd_variant<true>(b, w, frags, bal, grid, st);
  else
    raster_fwd_variant<false>(b, w, frags, bal, grid, st);
  return hipGetLastError();
}

template <int NV, bool GA>
static void raster_bwd_variant(const Batch& b, const WsPtrs& w, bool frags, bool bal, int grid,
                               hipStream_t st) {
  if (frags) {
    if (bal)
      k_raster_bwd<NV, GA, true, true, false><<<grid, kBlock, 0, st>>>(b, w);
    else
      k_raster_bwd<NV, GA, true, false, false><<<grid, kBlock, 0, st>>>(b, w);
  } else {
    if (bal)
      k_raster_bwd<NV, GA, false, true, false><<<grid, kBlock, 0, st>>>(b, w);
    else if (b.n_sessions == 1)
      k_raster_bwd<NV, GA, false, false, true><<<grid, kBlock, 0, st>>>(b, w);
    else
      k_raster_bwd<NV, GA, false, false, false><<<grid, kBlock, 0, st>>>(b, w);
  }
}

hipError_t launch_raster_bwd(const Batch& b, const WsPtrs& w, int pose_only, bool alpha_grad,
                             bool frags, bool bal, hipStream_t st, StageTimer* tm) {
  if (b.t_total <= 0) return hipGetLastError();
  const int grid = 8 * ((b.t_total + 7) / 8);
  Scope sc(tm, kStRasterBwd, st);
  if (pose_only) {
    if (alpha_grad)
      raster_bwd_variant<6, true>(b, w, frags, bal, grid, st);
    else
      raster_bwd_variant<6, false>(b, w, frags, bal, grid, st);
  } else {
    if (alpha_grad)
      raster_bwd_variant<10, true>(b, w, frags, bal, grid, st);
    else
      raster_bwd_variant<10, false>(b, w, frags, bal, grid, st);
  }
  return hipGetLastError();
}

}  // namespace rtgs
