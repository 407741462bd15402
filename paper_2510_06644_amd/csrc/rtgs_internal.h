// Internal declarations of librtgs: device-side session table, workspace
// layout, launch wrappers and the device helpers shared by the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/rtgs.h"

namespace rtgs {

constexpr int kTile = 16;                 // tile edge in pixels (Sec. 2.1)
constexpr int kBlock = 256;               // threads per workgroup
constexpr int kGaussPerBlock = 256;       // Gaussians per block, per-Gaussian kernels
constexpr float kAlphaMin = 1.0f / 255.0f;  // skip floor for a fragment
constexpr float kAlphaMax = 0.99f;          // alpha clamp
constexpr float kTMin = 1e-4f;              // early-termination transmittance
constexpr double kNearZ = 0.2;
constexpr double kDilation = 0.3;
constexpr double kFovClamp = 1.3;
constexpr int kChunk = 1024;              // Gaussians per binning chunk (1 per thread)
constexpr int kMaxTilesPerSession = 12288; // LDS tile histogram of one session (48 KB)

// Adam state of a session's map for an update fused into the backward
// (constants formed on the host as adam_step forms them).
struct MapAdamDev {
  float* m[5];            // first moments: means, log_scales, quats, opacity, colours
  float* v[5];            // second moments
  float step_size[5];     // lr / (1 - beta1^t)
  float inv_sqrt_bc2;     // 1 / sqrt(1 - beta2^t)
  float beta1, beta2, omb1, omb2, eps;
  int32_t on;
};

// Device copy of one session (built on the host from rtgs_session).
struct SessionDev {
  // map
  const float* means;
  const float* log_scales;
  const float* quats;
  const float* opac;
  const float* colors;
  const uint8_t* gmask;
  const float* viewmat;
  const uint8_t* pmask;
  // forward outputs
  float* color;
  float* depth;
  float* alpha;
  float* final_T;
  int32_t* last_idx;
  uint8_t* visible;
  int32_t* stats;       // [3][H][W] or null: blended, entries visited, entries to last
  const uint16_t* lane_work;  // [H][W] entries walked per sample in a previous forward, or null
  uint16_t* lane_work_out;    // [H][W] this forward's, or null
  // loss gradient written by the forward (l1_dcolor null: none)
  const float* l1_tcolor;
  const float* l1_tdepth;
  const int32_t* l1_n_active;
  float* l1_dcolor;
  float* l1_ddepth;
  float l1_w_color, l1_w_depth;
  // backward
  const float* dl_color;
  const float* dl_depth;
  const float* dl_alpha;
  float* g_means;
  float* g_log_scales;
  float* g_quats;
  float* g_opac;
  float* g_colors;
  float* g_pose6;
  float* g_viewmat;
  float* g_cov3d;
  MapAdamDev adam;      // RTGS_GRAD_ADAM: the map's update after its gradients
  // geometry
  int32_t n;
  int32_t width;
  int32_t height;
  int32_t tiles_x;
  int32_t tiles_y;
  int32_t sub_sx;       // log2 of the sample block width (0: one sample per pixel)
  int32_t sub_sy;       // log2 of the sample block height
  float fx, fy, cx, cy;
  // offsets into the batch-global index spaces
  int32_t gauss_base;   // first global Gaussian index
  int32_t block_base;   // first per-Gaussian block
  int32_t tile_base;    // first global tile
  int32_t chunk_base;   // first binning chunk
  int64_t hist_base;    // first entry of this session's [chunk][tile] counts
};

// Offsets of the workspace regions (bytes from ws).
struct WsLayout {
  uint64_t table;       // SessionDev[RTGS_MAX_SESSIONS]
  uint64_t counters;    // int64[8]: 0 pairs of this call, 2 entries of big_tiles
  uint64_t rec;         // GaussRec[N]: the 64-byte raster record of each Gaussian
  uint64_t rect;        // int4[N]: tile rectangle
  uint64_t cnt;         // uint32[N]: tiles touched
  uint64_t goff;        // uint32[N]: first slot of the Gaussian's pairs, Gaussian-major
  uint64_t zkey;        // uint32[N]: depth bits of the Gaussian's sort key (projection)
  uint64_t grad2d;      // float[N][10]: merged dL/d(u, v, a, b, c, o, r, g, b, z)
  uint64_t pose_part;   // double[B][16]: per-block view-matrix gradient partial sums
  uint64_t chunk_total; // uint32[C + 1]: pairs per chunk
  uint64_t chunk_off;   // uint32[C + 1]: exclusive scan of chunk_total
  uint64_t hist;        // uint32[sum_s C_s T_s]: per (chunk, tile) counts, then each
                        // chunk's exclusive scan over its tiles (run offsets in the chunk)
  uint64_t gsum;        // uint32[16][T]: per (group of chunks, tile) sums
  uint64_t tile_count;  // uint32[T + 1]
  uint64_t tile_start;  // uint32[T + 1]
  uint64_t big_tiles;   // uint32[T]: tiles whose list is too long for the one-pass sort
  uint64_t keys;        // uint64[cap]: (depth bits << 32 | id), chunk-major
  uint64_t keys_tm;     // uint64[cap]: the long lists gathered tile-major for their sort
  uint64_t ids;         // uint32[cap]
  uint64_t qmask;       // uint8[cap]: quadrants of its tile each list entry can reach
  uint64_t partial;     // float[cap][10]: per (tile, Gaussian) merged 2D gradient
  uint64_t state_t;     // float[pixels]: recomputed final T
  uint64_t state_last;  // int32[pixels]: recomputed last position
  uint64_t lane_perm;   // uint8[T][256]: sample of each lane (lanes assigned by previous work)
  // saved fragments (workspace sized with RTGS_FWD_SAVE_FRAGMENTS, else absent)
  uint64_t fmask;       // uint64[4 cap]: blend mask of each (list entry, wave)
  uint64_t fcount;      // uint32[4 T]: saved fragments of each (tile, wave)
  uint64_t fdata;       // float2[256 cap]: (alpha, 1 - alpha) streams per (tile, wave)
  uint64_t total;       // bytes
  int64_t n_total;
  int64_t t_total;
  int64_t b_total;
  int64_t cap;
};

struct Counts {
  int64_t n_total = 0, t_total = 0, b_total = 0, c_total = 0, h_total = 0, px_total = 0;
  int64_t t_max = 0;
};

WsLayout make_layout(const Counts& c, int64_t cap, bool frags = false);

// What the raster kernels read of one Gaussian, packed into one 64-byte
// line so that staging a list entry touches a single cache line.
struct alignas(64) GaussRec {
  float4 pos;     // u_hi, v_hi, u_lo, v_lo (centre as a float32 pair)
  float4 conic;   // a, b, c (inverse 2D covariance), opacity
  float4 col;     // r, g, b, depth z
  float4 ext;     // e_x, e_y (half-widths of the alpha = 1/255 box), t = 2 ln(255 o), 0
};
static_assert(sizeof(GaussRec) == 64, "one line per record");

// Pointers derived from a workspace.
struct WsPtrs {
  SessionDev* table;
  long long* counters;
  GaussRec* rec;
  int4* rect;
  uint32_t* cnt;
  uint32_t* goff;
  uint32_t* zkey;
  float* grad2d;
  double* pose_part;
  uint32_t* chunk_total;
  uint32_t* chunk_off;
  uint32_t* hist;
  uint32_t* gsum;
  uint32_t* tile_count;
  uint32_t* tile_start;
  uint32_t* big_tiles;
  unsigned long long* keys;
  unsigned long long* keys_tm;
  uint32_t* ids;
  uint8_t* qmask;
  float* partial;
  float* state_t;
  int32_t* state_last;
  uint8_t* lane_perm;
  unsigned long long* fmask;   // null without saved fragments
  uint32_t* fcount;
  float2* fdata;
  int64_t cap;
};

WsPtrs ws_ptrs(void* ws, const WsLayout& L);

// Batch geometry passed by value to every kernel.
struct Batch {
  const SessionDev* sess;   // device session table (read when n_sessions > 1)
  int32_t n_sessions;
  int32_t n_total;      // Gaussians over all sessions
  int32_t t_total;      // tiles over all sessions
  int32_t b_total;      // per-Gaussian blocks over all sessions
  int32_t c_total;      // binning chunks over all sessions
  int32_t t_max;        // largest tile count of one session
  SessionDev one;       // the session of a one-session batch, passed with the launch
                        // arguments instead of through a table upload
};

// Stages that the handle's profiler can bracket with HIP events.
enum Stage {
  kStInit = 0, kStPreprocess, kStScan, kStEmit, kStSort, kStRasterFwd, kStAdam, kStRasterBwd,
  kStPreprocessBwd, kStPoseReduce, kStBinCount, kStMerge, kStCount
};

// Records HIP events around kernel launches of the enabled stages.
struct StageTimer {
  virtual void begin(int stage, hipStream_t st) = 0;
  virtual void end(int stage, hipStream_t st) = 0;
  virtual ~StageTimer() = default;
};

struct Scope {
  StageTimer* t;
  int stage;
  hipStream_t st;
  Scope(StageTimer* t_, int s_, hipStream_t st_) : t(t_), stage(s_), st(st_) {
    if (t) t->begin(stage, st);
  }
  ~Scope() {
    if (t) t->end(stage, st);
  }
};

// ---- launch wrappers (defined in the .hip files) ----
hipError_t launch_forward_prep(const Batch& b, const WsPtrs& w, unsigned long long* max_pairs,
                               bool reuse_lists, hipStream_t st, StageTimer* tm);
hipError_t launch_raster_fwd(const Batch& b, const WsPtrs& w, bool stats, bool frags, bool bal,
                             hipStream_t st, StageTimer* tm);
hipError_t launch_raster_bwd(const Batch& b, const WsPtrs& w, int pose_only, bool alpha_grad,
                             bool frags, bool bal, hipStream_t st, StageTimer* tm);
hipError_t launch_preprocess_bwd(const Batch& b, const WsPtrs& w, int grad_flags, hipStream_t st,
                                 StageTimer* tm);
hipError_t launch_prune(const float* g_means, const float* g_cov3d, const uint8_t* visible,
                        const uint8_t* mask_in, int n, float lambda, float ratio,
                        uint8_t* mask_out, int* n_masked, float* score_out, uint32_t* scratch,
                        hipStream_t st);
hipError_t launch_downsample(const float* final_T, int w, int h, int j, uint8_t* mask_out,
                             int* n_active, hipStream_t st);
hipError_t launch_debug_stage(const Batch& b, const WsPtrs& w, float* stage, int* rect,
                              int* ranges, int* ids, int64_t ids_cap, hipStream_t st);
hipError_t launch_wave_sum_test(const float* in, float* out, int n_waves, hipStream_t st);
constexpr int kWaveSumValues = 10;    // values per lane in the reduction self-test

// One Adam update over up to kAdamMaxGroups parameter tensors in one launch.
constexpr int kAdamMaxGroups = 64;
struct AdamGroupDev {
  float* p;
  const float* g;
  float* m;
  float* v;
  int64_t n;
  float step_size;      // lr / (1 - beta1^t)
  float inv_sqrt_bc2;   // 1 / sqrt(1 - beta2^t)
  int32_t vec;          // all four arrays 16-byte aligned
  int32_t block0;       // first block of the group
};
struct AdamArgs {
  AdamGroupDev grp[kAdamMaxGroups];
  int32_t n_groups;
  int32_t n_blocks;
  float beta1, beta2, omb1, omb2, eps;   // omb = 1 - beta, rounded once from double
};
hipError_t launch_adam(const AdamArgs& a, hipStream_t st, StageTimer* tm);

struct LossArgs {
  const float* color;     // [3][H][W]
  const float* depth;     // [H][W]
  const float* t_color;
  const float* t_depth;
  const uint8_t* mask;    // [H][W] or null
  const int32_t* n_active;  // device count of active pixels, or null (H * W)
  float* g_color;
  float* g_depth;
  int32_t w, h;
  float w_color, w_depth;
};
hipError_t launch_l1_grad(const LossArgs& a, hipStream_t st);

// Several frames' loss gradients in one launch (up to kLossMaxItems).
constexpr int kLossMaxItems = 32;
struct LossItemDev {
  LossArgs a;
  int32_t block_base;       // first block of this item
};
struct LossBatchArgs {
  LossItemDev item[kLossMaxItems];
  int32_t n;
};
hipError_t launch_l1_grad_batched(const LossBatchArgs& a, int total_blocks, hipStream_t st);

// Pose update of up to kPoseMaxItems sessions in one launch.
constexpr int kPoseMaxItems = 48;
struct PoseItemDev {
  float* viewmat;         // [12] row-major 3x4, updated in place
  const float* g_pose6;   // [6] dL/d(rho, phi)
  float* exp_avg;         // [6]
  float* exp_avg_sq;      // [6]
  double lr_rho, lr_phi;
  double bc1, bc2;        // 1 - beta1^t, 1 - beta2^t
};
struct PoseArgs {
  PoseItemDev item[kPoseMaxItems];
  int32_t n;
  double beta1, beta2, eps;
};
hipError_t launch_pose_update(const PoseArgs& a, hipStream_t st);
constexpr int kAdamPerThread = 4;

constexpr int kPruneScratchWords = 4096;

// Stable compaction of per-Gaussian arrays by a drop mask (the permanent
// removal of the mask-prune schedule).
constexpr int kCompactMaxItems = 24;
constexpr int kCompactBlock = 1024;
struct CompactItemDev {
  const unsigned char* src;
  unsigned char* dst;
  int32_t row_bytes;
  int32_t dst_rows;
};
struct CompactArgs {
  CompactItemDev item[kCompactMaxItems];
  int32_t n_items;
  int32_t n;
  const uint8_t* drop;
  uint32_t* block_keep;    // [ceil(n / kCompactBlock) + 1] scratch
  int32_t* n_kept;
};
hipError_t launch_compact(const CompactArgs& a, hipStream_t st);
// Words of compact_by_mask_static's device scratch, and its address on the
// current GPU (taken once per GPU; no allocation).
constexpr int kCompactStaticWords = 16384;
hipError_t compact_static_scratch(uint32_t** out);
hipError_t launch_rect_change(const int32_t* a, const int32_t* b, const uint8_t* skip, int n,
                              int64_t* out, hipStream_t st);

// ---- device helpers ----
#if defined(__HIP_DEVICE_COMPILE__) || defined(__HIPCC__)

// Session owning a block, by binary search over a monotone base field.
template <typename F>
__device__ __forceinline__ int find_session(const SessionDev* s, int n, int key, F base) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (base(s[mid]) <= key) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Sign of the L1 loss derivative: 1, -1, or 0 where the residual is 0.
__device__ __forceinline__ float sign_of(float x) {
  return x > 0.f ? 1.f : (x < 0.f ? -1.f : 0.f);
}

// Session s of a batch.
__device__ __forceinline__ const SessionDev& session_of(const Batch& B, int s) {
  return B.n_sessions == 1 ? B.one : B.sess[s];
}

// The device session table seen through the constant address space: the
// kernels never write it, and read through such a pointer its uniform fields
// become scalar loads (through session_of's reference, which may point into
// the launch arguments or the table, each is a vector load that waits behind
// every earlier store).  Valid when the host uploaded the table (see
// batch_session).
__device__ __forceinline__ const SessionDev* session_table(const Batch& B) {
  typedef const __attribute__((address_space(4))) SessionDev ConstSession;
  return (const SessionDev*)(ConstSession*)B.sess;
}

// Session s of a batch, for kernels instantiated per batch kind.  ONE (the
// host launches it only for a batch of one session): the session is read
// from the launch arguments.  Otherwise from the table, which the host then
// uploads (also for one session).  Either way its fields are read with scalar
// loads.
template <bool ONE>
__device__ __forceinline__ const SessionDev& batch_session(const Batch& B, int s) {
  return ONE ? B.one : session_table(B)[s];
}

// DPP control words (GFX9 encoding).
constexpr int kDppRowShr1 = 0x111;
constexpr int kDppRowShr2 = 0x112;
constexpr int kDppRowShr4 = 0x114;
constexpr int kDppRowShr8 = 0x118;
constexpr int kDppRowBcast15 = 0x142;
constexpr int kDppRowBcast31 = 0x143;

template <int CTRL, int ROW_MASK, bool BOUND_ZERO>
__device__ __forceinline__ float dpp_f(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(
      0, __builtin_bit_cast(int, v), CTRL, ROW_MASK, 0xf, BOUND_ZERO));
}

// Sum of a 16-lane row, inclusive scan by shifted adds (out-of-row sources
// read 0): lane 15 of each row ends with the row total.
__device__ __forceinline__ float row_sum_to_lane15(float v) {
  v += dpp_f<kDppRowShr1, 0xf, true>(v);
  v += dpp_f<kDppRowShr2, 0xf, true>(v);
  v += dpp_f<kDppRowShr4, 0xf, true>(v);
  v += dpp_f<kDppRowShr8, 0xf, true>(v);
  // keep the last step a single DPP add in every lane: otherwise the add is
  // sunk into the caller's lane-15-only branch as a separate move and add
  asm volatile("" : "+v"(v));
  return v;
}

// a + b for a pair of registers after v_permlane32_swap: lanes 0-31 get
// a(l) + a(l + 32), lanes 32-63 get b(l - 32) + b(l).
__device__ __forceinline__ float swap32_add(float a, float b) {
  // (the two results are copied out as integers first: a bit cast applied
  // to an element of the returned pair reads the first element for both)
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false,
                                                  false);
  const unsigned x = r[0], y = r[1];
  return __uint_as_float(x) + __uint_as_float(y);
}

// The same with v_permlane16_swap between rows 2i and 2i + 1 (16 lanes each):
// row 2i gets a summed over both rows, row 2i + 1 gets b summed over both.
__device__ __forceinline__ float swap16_add(float a, float b) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false,
                                                  false);
  const unsigned x = r[0], y = r[1];
  return __uint_as_float(x) + __uint_as_float(y);
}

// Wavefront reduce-scatter of NV (even, <= 12) per-lane values.  Two
// lane-swap steps each halve the number of values a lane carries while
// adding pairs of lanes; the (at most 3) values left are then summed along
// each 16-lane row.  With NV / 2 odd, the last value after the first swap has
// no partner for the second: it is summed along each row as it is, and the
// total of row 2i is added into row 2i + 1 by a row broadcast.  Lane 16 r + 15
// (row r) ends with, in x[s], the wavefront total of value
// wave_scatter_index(NV, r, s) where that is >= 0.  About 3 NV instructions
// instead of the 6 NV of a full tree per value.
template <int NV>
__device__ __forceinline__ void wave_reduce_scatter(const float (&v)[NV], float (&x)[3]) {
  constexpr int H = NV / 2;
  static_assert(NV % 2 == 0 && H <= 6, "even value count up to 12");
  float w[H];
#pragma unroll
  for (int i = 0; i < H; ++i) w[i] = swap32_add(v[i], v[i + H]);
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    if (2 * j + 1 < H) {
      x[j] = row_sum_to_lane15(swap16_add(w[2 * j], w[2 * j + 1]));
    } else if (2 * j < H) {
      x[j] = row_sum_to_lane15(w[2 * j]);
      // rows 1 and 3 add lane 15 of rows 0 and 2 (even rows end with
      // something meaningless, which wave_scatter_index excludes)
      x[j] += dpp_f<kDppRowBcast15, 0xf, true>(x[j]);
      asm volatile("" : "+v"(x[j]));   // one DPP add in every lane (see above)
    } else {
      x[j] = 0.f;
    }
  }
}

// The value whose total lane 16 row + 15 holds in x[s] after
// wave_reduce_scatter<NV>, or -1 if that output carries none.
__device__ __forceinline__ int wave_scatter_index(int nv, int row, int s) {
  const int h = nv / 2;
  if (2 * s + 1 < h) return (row >> 1) * h + (row & 1) + 2 * s;
  if (2 * s < h) return (row & 1) ? (row >> 1) * h + 2 * s : -1;
  return -1;
}

// One Adam element update (t the step count after it):
//   m <- beta1 m + (1 - beta1) g,  v <- beta2 v + (1 - beta2) g^2,
//   p <- p - (lr / (1 - beta1^t)) m / (sqrt(v) / sqrt(1 - beta2^t) + eps).
__device__ __forceinline__ void adam_update(float& p, float g, float& m, float& v, float beta1,
                                            float beta2, float omb1, float omb2, float eps,
                                            float step, float isb2) {
  m = __builtin_fmaf(omb1, g, beta1 * m);
  v = __builtin_fmaf(omb2, g * g, beta2 * v);
  const float denom = __builtin_fmaf(__builtin_sqrtf(v), isb2, eps);
  p = p - step * (m / denom);
}

// Activations of Eq. 1's parameters (scales exp(l), opacity sigmoid(eta)),
// evaluated in float32 from the float32 parameters (about 1e-7 relative, far
// inside the float32 rendering) and widened for the float64 projection: the
// float64 exp is a long software routine on the GPU.
__device__ __forceinline__ void activate(const SessionDev& S, int li, double (&sc)[3], double& o) {
#pragma unroll
  for (int k = 0; k < 3; ++k) sc[k] = (double)expf(S.log_scales[3 * li + k]);
  o = (double)(1.f / (1.f + expf(-S.opac[li])));
}

// Raster-side alpha of one (pixel, Gaussian) pair: the same instructions in
// the forward and the backward so both take the same skip decisions.
// r0 = (u_hi, v_hi, u_lo, v_lo); k = (A, B, C, opacity), the conic (a, b, c)
// pre-scaled to base-2 exponent units by conic_log2(), so that
// exp(power) = 2^(A dx^2 + B dx dy + C dy^2) is one v_exp_f32.
struct Frag {
  float dx, dy, e, alpha;   // e = exp(power), alpha = min(0.99, o e)
  float om;                 // 1 - alpha, from one fused rounding of 1 - o e
};

constexpr float kLog2e = 1.4426950408889634f;

// (a, b, c, o) -> (-a log2(e) / 2, -b log2(e), -c log2(e) / 2, o):
// power = -(a dx^2 + 2 b dx dy + c dy^2) / 2 in natural-log units.
__device__ __forceinline__ float4 conic_log2(float4 c) {
  return make_float4(-0.5f * kLog2e * c.x, -kLog2e * c.y, -0.5f * kLog2e * c.z, c.w);
}

__device__ __forceinline__ Frag frag_alpha(float4 r0, float4 k, float px, float py) {
  Frag f;
  f.dx = (r0.x - px) + r0.z;
  f.dy = (r0.y - py) + r0.w;
  // log2 of exp(power) = dx (A dx + B dy) + C dy^2
  const float t = __builtin_fmaf(k.x, f.dx, k.y * f.dy);
  const float p2 = __builtin_fmaf(f.dx, t, (k.z * f.dy) * f.dy);
  f.e = __builtin_amdgcn_exp2f(p2);
  const float raw = k.w * f.e;
  f.alpha = fminf(kAlphaMax, raw);
  // 1 - alpha without rounding o e first: near-opaque fragments (alpha close
  // to 0.99) would otherwise lose digits of the transmittance they leave
  // (clamped: 1 - o e < 1 - 0.99, so the max gives 1 - 0.99 up to one rounding)
  f.om = fmaxf(1.f - kAlphaMax, __builtin_fmaf(-k.w, f.e, 1.f));
  return f;
}

#endif

}  // namespace rtgs
