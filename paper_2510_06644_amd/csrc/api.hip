// Host side of the C ABI declared in include/rtgs.h: argument validation,
// workspace layout, the device session table and the launch sequence.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "rtgs_internal.h"

using namespace rtgs;

namespace {

thread_local std::string g_err = "no error";

int32_t fail(int32_t code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int32_t hip_fail(hipError_t e, const char* what) {
  return fail(RTGS_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

constexpr int kRing = 16;
constexpr uint64_t kAlign = 256;

uint64_t align_up(uint64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Sample block of a downsampled frame: 2^ceil(j/2) x 2^floor(j/2) pixels.
int sub_sx(int j) { return (j + 1) / 2; }
int sub_sy(int j) { return j / 2; }

int64_t tiles_of(int w, int h, int j = 0) {
  const int tw = kTile << sub_sx(j), th = kTile << sub_sy(j);
  return (int64_t)((w + tw - 1) / tw) * ((h + th - 1) / th);
}

int64_t blocks_of(int n) { return (n + kGaussPerBlock - 1) / kGaussPerBlock; }

int64_t chunks_of(int n) { return (n + kChunk - 1) / kChunk; }

}  // namespace

namespace {

// HIP-event stage timer owned by a handle.
struct EventTimer : StageTimer {
  int mask = 0;
  std::vector<hipEvent_t> pool;
  struct Rec {
    int stage;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  std::vector<int> open_stage;
  std::vector<hipEvent_t> open_ev;
  hipError_t err = hipSuccess;

  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    hipError_t r = hipEventCreate(&e);
    if (r != hipSuccess) err = r;
    return e;
  }
  void begin(int stage, hipStream_t st) override {
    if (!(mask & (1 << stage))) return;
    hipEvent_t e = get();
    if (e && hipEventRecord(e, st) != hipSuccess) err = hipErrorUnknown;
    open_stage.push_back(stage);
    open_ev.push_back(e);
  }
  void end(int stage, hipStream_t st) override {
    if (!(mask & (1 << stage))) return;
    hipEvent_t e = get();
    if (e && hipEventRecord(e, st) != hipSuccess) err = hipErrorUnknown;
    hipEvent_t a = open_ev.back();
    open_ev.pop_back();
    open_stage.pop_back();
    recs.push_back({stage, a, e});
  }
  ~EventTimer() override {
    for (auto& r : recs) {
      (void)hipEventDestroy(r.a);
      (void)hipEventDestroy(r.b);
    }
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

}  // namespace

struct rtgs_context {
  int device = 0;
  EventTimer timer;
  unsigned long long* d_scalars = nullptr;   // [0] largest pair count since last query,
                                             // [1] largest count that overflowed (or 0)
  uint32_t* d_prune = nullptr;               // prune scratch
  SessionDev* h_ring = nullptr;              // pinned [kRing][RTGS_MAX_SESSIONS]
  hipEvent_t ring_ev[kRing] = {};
  int ring_pos = 0;
  hipStream_t last_stream = nullptr;
  bool used = false;
};

namespace rtgs {

WsLayout make_layout(const Counts& c, int64_t cap, bool frags) {
  WsLayout L{};
  uint64_t off = 0;
  auto take = [&](uint64_t bytes) {
    const uint64_t at = off;
    off = align_up(off + bytes);
    return at;
  };
  const uint64_t n = (uint64_t)c.n_total, t = (uint64_t)c.t_total;
  L.table = take(sizeof(SessionDev) * RTGS_MAX_SESSIONS);
  L.counters = take(64);
  L.rec = take(64 * n);
  L.rect = take(16 * n);
  L.cnt = take(4 * n);
  L.goff = take(4 * n);
  L.zkey = take(4 * n);
  L.grad2d = take(40 * n);
  L.pose_part = take(128 * (uint64_t)c.b_total);
  L.chunk_total = take(4 * (uint64_t)(c.c_total + 1));
  L.chunk_off = take(4 * (uint64_t)(c.c_total + 1));
  L.hist = take(4 * (uint64_t)c.h_total);
  L.gsum = take(4 * 16 * t);
  L.tile_count = take(4 * (t + 1));
  L.tile_start = take(4 * (t + 1));
  L.big_tiles = take(4 * (t + 1));
  L.keys = take(8 * (uint64_t)cap);
  L.keys_tm = take(8 * (uint64_t)cap);
  L.ids = take(4 * (uint64_t)cap);
  L.qmask = take((uint64_t)cap);
  L.partial = take(4 * 10 * (uint64_t)cap);
  L.state_t = take(4 * (uint64_t)c.px_total);
  L.state_last = take(4 * (uint64_t)c.px_total);
  L.lane_perm = take(256 * t);
  if (frags) {
    L.fmask = take(8 * 4 * (uint64_t)cap);
    L.fcount = take(4 * 4 * t);
    L.fdata = take(8 * 256 * (uint64_t)cap);
  }
  L.total = off;
  L.n_total = c.n_total;
  L.t_total = c.t_total;
  L.b_total = c.b_total;
  L.cap = cap;
  return L;
}

WsPtrs ws_ptrs(void* ws, const WsLayout& L) {
  char* base = static_cast<char*>(ws);
  WsPtrs w{};
  w.table = reinterpret_cast<SessionDev*>(base + L.table);
  w.counters = reinterpret_cast<long long*>(base + L.counters);
  w.rec = reinterpret_cast<GaussRec*>(base + L.rec);
  w.rect = reinterpret_cast<int4*>(base + L.rect);
  w.cnt = reinterpret_cast<uint32_t*>(base + L.cnt);
  w.goff = reinterpret_cast<uint32_t*>(base + L.goff);
  w.zkey = reinterpret_cast<uint32_t*>(base + L.zkey);
  w.grad2d = reinterpret_cast<float*>(base + L.grad2d);
  w.pose_part = reinterpret_cast<double*>(base + L.pose_part);
  w.chunk_total = reinterpret_cast<uint32_t*>(base + L.chunk_total);
  w.chunk_off = reinterpret_cast<uint32_t*>(base + L.chunk_off);
  w.hist = reinterpret_cast<uint32_t*>(base + L.hist);
  w.gsum = reinterpret_cast<uint32_t*>(base + L.gsum);
  w.tile_count = reinterpret_cast<uint32_t*>(base + L.tile_count);
  w.tile_start = reinterpret_cast<uint32_t*>(base + L.tile_start);
  w.big_tiles = reinterpret_cast<uint32_t*>(base + L.big_tiles);
  w.keys = reinterpret_cast<unsigned long long*>(base + L.keys);
  w.keys_tm = reinterpret_cast<unsigned long long*>(base + L.keys_tm);
  w.ids = reinterpret_cast<uint32_t*>(base + L.ids);
  w.qmask = reinterpret_cast<uint8_t*>(base + L.qmask);
  w.partial = reinterpret_cast<float*>(base + L.partial);
  w.state_t = reinterpret_cast<float*>(base + L.state_t);
  w.state_last = reinterpret_cast<int32_t*>(base + L.state_last);
  w.lane_perm = reinterpret_cast<uint8_t*>(base + L.lane_perm);
  if (L.fdata) {
    w.fmask = reinterpret_cast<unsigned long long*>(base + L.fmask);
    w.fcount = reinterpret_cast<uint32_t*>(base + L.fcount);
    w.fdata = reinterpret_cast<float2*>(base + L.fdata);
  }
  w.cap = L.cap;
  return w;
}

}  // namespace rtgs

namespace {

int32_t geometry(const int32_t* n, const int32_t* w, const int32_t* h, int32_t ns, Counts& g,
                 const int32_t* js = nullptr) {
  if (ns < 1 || ns > RTGS_MAX_SESSIONS)
    return fail(RTGS_ERR_INVALID_ARG, "n_sessions %d outside [1, %d]", ns, RTGS_MAX_SESSIONS);
  for (int s = 0; s < ns; ++s) {
    if (n[s] < 0) return fail(RTGS_ERR_INVALID_ARG, "session %d: n = %d < 0", s, n[s]);
    if (w[s] <= 0 || h[s] <= 0)
      return fail(RTGS_ERR_INVALID_ARG, "session %d: image %d x %d", s, w[s], h[s]);
    const int j = js ? js[s] : 0;
    if (j < 0 || j > 4)
      return fail(RTGS_ERR_INVALID_ARG, "session %d: sample_log2 %d outside [0, 4]", s, j);
    const int64_t t = tiles_of(w[s], h[s], j);
    if (t > kMaxTilesPerSession)
      return fail(RTGS_ERR_INVALID_ARG, "session %d: %lld tiles > %d (image too large)", s,
                  (long long)t, kMaxTilesPerSession);
    g.n_total += n[s];
    g.t_total += t;
    g.b_total += blocks_of(n[s]);
    g.c_total += chunks_of(n[s]);
    g.h_total += chunks_of(n[s]) * t;
    g.px_total += (int64_t)w[s] * h[s];
    if (t > g.t_max) g.t_max = t;
  }
  if (g.n_total > INT32_MAX / 2 || g.t_total > INT32_MAX / 2 || g.px_total > INT32_MAX / 2 ||
      g.h_total > INT32_MAX)
    return fail(RTGS_ERR_INVALID_ARG, "batch too large");
  return RTGS_OK;
}

int32_t check_cap(int64_t cap) {
  if (cap < 0 || cap > (int64_t)INT32_MAX)
    return fail(RTGS_ERR_INVALID_ARG, "pair_capacity %lld outside [0, 2^31)", (long long)cap);
  return RTGS_OK;
}

// Validate one session's pointers for the requested direction.
int32_t check_session(const rtgs_session& s, int idx, bool fwd, int32_t flags) {
  const rtgs_gaussians& g = s.g;
  if (g.n > 0 && (!g.means || !g.log_scales || !g.quats || !g.opacity_logits || !g.colors))
    return fail(RTGS_ERR_INVALID_ARG, "session %d: null Gaussian parameter array", idx);
  if (!s.cam.viewmat) return fail(RTGS_ERR_INVALID_ARG, "session %d: null viewmat", idx);
  if (!(s.cam.fx > 0.f) || !(s.cam.fy > 0.f) || !std::isfinite(s.cam.fx) ||
      !std::isfinite(s.cam.fy) || !std::isfinite(s.cam.cx) || !std::isfinite(s.cam.cy))
    return fail(RTGS_ERR_INVALID_ARG, "session %d: bad intrinsics", idx);
  if (fwd) {
    if (!s.color || !s.depth || !s.alpha)
      return fail(RTGS_ERR_INVALID_ARG, "session %d: null colour/depth/alpha output", idx);
    if ((flags & RTGS_FWD_SAVE_STATE) && (!s.final_T || !s.last_idx))
      return fail(RTGS_ERR_INVALID_ARG, "session %d: SAVE_STATE needs final_T and last_idx", idx);
    if (s.l1) {
      const rtgs_l1_loss& l = *s.l1;
      if (!l.target_color || !l.target_depth || !l.dL_dcolor || !l.dL_ddepth)
        return fail(RTGS_ERR_INVALID_ARG, "session %d: null loss array", idx);
      if (s.pixel_mask && !l.n_active_dev)
        return fail(RTGS_ERR_INVALID_ARG, "session %d: loss with a pixel mask needs n_active_dev",
                    idx);
      if (!std::isfinite(l.w_color) || !std::isfinite(l.w_depth))
        return fail(RTGS_ERR_INVALID_ARG, "session %d: loss weights not finite", idx);
    }
  } else {
    if (!s.dL_dcolor || !s.dL_ddepth)
      return fail(RTGS_ERR_INVALID_ARG, "session %d: null dL/dcolor or dL/ddepth", idx);
    if (!(flags & RTGS_GRAD_RECOMPUTE_STATE) && (!s.final_T || !s.last_idx))
      return fail(RTGS_ERR_INVALID_ARG, "session %d: saved state missing", idx);
    if ((flags & RTGS_GRAD_MAP) && !(flags & RTGS_GRAD_ADAM) && g.n > 0 &&
        (!s.g_means || !s.g_log_scales || !s.g_quats || !s.g_opacity_logits || !s.g_colors))
      return fail(RTGS_ERR_INVALID_ARG, "session %d: null map gradient output", idx);
    if ((flags & RTGS_GRAD_ADAM) && s.adam) {
      const rtgs_map_adam& a = *s.adam;
      for (int k = 0; k < 5; ++k) {
        if (g.n > 0 && (!a.exp_avg[k] || !a.exp_avg_sq[k]))
          return fail(RTGS_ERR_INVALID_ARG, "session %d: null Adam moment array", idx);
        if (!std::isfinite(a.lr[k]))
          return fail(RTGS_ERR_INVALID_ARG, "session %d: Adam lr not finite", idx);
      }
      if (a.step < 1) return fail(RTGS_ERR_INVALID_ARG, "session %d: Adam step < 1", idx);
      if (!(a.beta1 >= 0.0 && a.beta1 < 1.0 && a.beta2 >= 0.0 && a.beta2 < 1.0))
        return fail(RTGS_ERR_INVALID_ARG, "session %d: Adam betas outside [0, 1)", idx);
      if (!(a.eps >= 0.0) || !std::isfinite(a.eps))
        return fail(RTGS_ERR_INVALID_ARG, "session %d: Adam eps must be finite and >= 0", idx);
    }
    if ((flags & RTGS_GRAD_POSE) && !s.g_pose6 && !s.g_viewmat)
      return fail(RTGS_ERR_INVALID_ARG, "session %d: POSE needs g_pose6 and/or g_viewmat", idx);
    if ((flags & RTGS_GRAD_COV3D) && (!(flags & RTGS_GRAD_MAP) || (g.n > 0 && !s.g_cov3d)))
      return fail(RTGS_ERR_INVALID_ARG, "session %d: COV3D needs MAP and g_cov3d", idx);
    if ((flags & RTGS_GRAD_SCORE) && !(flags & RTGS_GRAD_MAP) && (!s.g_means != !s.g_cov3d))
      return fail(RTGS_ERR_INVALID_ARG, "session %d: SCORE takes both g_means and g_cov3d "
                  "(or neither, to skip the session)", idx);
  }
  return RTGS_OK;
}

// Fill a ring slot with the device table, copy it into the workspace.
int32_t upload_table(rtgs_handle_t h, const rtgs_session* ss, int ns, const WsPtrs& w,
                     hipStream_t st, bool fwd, int32_t flags, Batch& B) {
  const int slot = h->ring_pos;
  h->ring_pos = (h->ring_pos + 1) % kRing;
  hipError_t e = hipEventSynchronize(h->ring_ev[slot]);
  if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
  SessionDev* t = h->h_ring + (size_t)slot * RTGS_MAX_SESSIONS;
  int32_t gbase = 0, bbase = 0, tbase = 0, cbase = 0, tmax = 0;
  int64_t pbase = 0, hbase = 0;
  for (int i = 0; i < ns; ++i) {
    const rtgs_session& s = ss[i];
    SessionDev d{};
    d.means = s.g.means;
    d.log_scales = s.g.log_scales;
    d.quats = s.g.quats;
    d.opac = s.g.opacity_logits;
    d.colors = s.g.colors;
    d.gmask = s.g.gauss_mask;
    d.viewmat = s.cam.viewmat;
    d.pmask = s.pixel_mask;
    d.n = s.g.n;
    d.width = s.cam.width;
    d.height = s.cam.height;
    d.sub_sx = sub_sx(s.sample_log2);
    d.sub_sy = sub_sy(s.sample_log2);
    d.tiles_x = (s.cam.width + (kTile << d.sub_sx) - 1) / (kTile << d.sub_sx);
    d.tiles_y = (s.cam.height + (kTile << d.sub_sy) - 1) / (kTile << d.sub_sy);
    d.fx = s.cam.fx;
    d.fy = s.cam.fy;
    d.cx = s.cam.cx;
    d.cy = s.cam.cy;
    d.gauss_base = gbase;
    d.block_base = bbase;
    d.tile_base = tbase;
    d.chunk_base = cbase;
    d.hist_base = hbase;
    if (fwd) {
      d.color = s.color;
      d.depth = s.depth;
      d.alpha = s.alpha;
      d.final_T = (flags & RTGS_FWD_SAVE_STATE) ? s.final_T : nullptr;
      d.last_idx = (flags & RTGS_FWD_SAVE_STATE) ? s.last_idx : nullptr;
      d.visible = s.visible;
      d.stats = (flags & RTGS_FWD_STATS) ? s.stats : nullptr;
      d.lane_work = (flags & RTGS_FWD_BALANCE_LANES) ? s.lane_work : nullptr;
      d.lane_work_out = (flags & RTGS_FWD_BALANCE_LANES) ? s.lane_work_out : nullptr;
      if (s.l1) {
        d.l1_tcolor = s.l1->target_color;
        d.l1_tdepth = s.l1->target_depth;
        d.l1_n_active = s.l1->n_active_dev;
        d.l1_dcolor = s.l1->dL_dcolor;
        d.l1_ddepth = s.l1->dL_ddepth;
        d.l1_w_color = s.l1->w_color;
        d.l1_w_depth = s.l1->w_depth;
      }
    } else {
      if (flags & RTGS_GRAD_RECOMPUTE_STATE) {
        d.final_T = w.state_t + pbase;
        d.last_idx = w.state_last + pbase;
      } else {
        d.final_T = const_cast<float*>(s.final_T);
        d.last_idx = const_cast<int32_t*>(s.last_idx);
      }
      d.dl_color = s.dL_dcolor;
      d.dl_depth = s.dL_ddepth;
      d.dl_alpha = s.dL_dalpha;
      if (flags & RTGS_GRAD_MAP) {
        d.g_means = s.g_means;
        d.g_log_scales = s.g_log_scales;
        d.g_quats = s.g_quats;
        d.g_opac = s.g_opacity_logits;
        d.g_colors = s.g_colors;
        d.g_cov3d = (flags & RTGS_GRAD_COV3D) ? s.g_cov3d : nullptr;
      } else if (flags & RTGS_GRAD_SCORE) {
        d.g_means = s.g_means;
        d.g_cov3d = s.g_cov3d;
      }
      if ((flags & RTGS_GRAD_ADAM) && s.adam) {
        // the constants adam_step forms, so the two updates agree bitwise
        const rtgs_map_adam& a = *s.adam;
        MapAdamDev& m = d.adam;
        for (int k = 0; k < 5; ++k) {
          m.m[k] = a.exp_avg[k];
          m.v[k] = a.exp_avg_sq[k];
          m.step_size[k] = (float)((double)a.lr[k] / (1.0 - std::pow(a.beta1, (double)a.step)));
        }
        m.inv_sqrt_bc2 = (float)(1.0 / std::sqrt(1.0 - std::pow(a.beta2, (double)a.step)));
        m.beta1 = (float)a.beta1;
        m.beta2 = (float)a.beta2;
        m.omb1 = (float)(1.0 - a.beta1);
        m.omb2 = (float)(1.0 - a.beta2);
        m.eps = (float)a.eps;
        m.on = 1;
      }
      d.g_pose6 = (flags & RTGS_GRAD_POSE) ? s.g_pose6 : nullptr;
      d.g_viewmat = (flags & RTGS_GRAD_POSE) ? s.g_viewmat : nullptr;
    }
    t[i] = d;
    gbase += s.g.n;
    bbase += (int32_t)blocks_of(s.g.n);
    const int32_t ts = (int32_t)tiles_of(s.cam.width, s.cam.height, s.sample_log2);
    tbase += ts;
    cbase += (int32_t)chunks_of(s.g.n);
    hbase += chunks_of(s.g.n) * ts;
    if (ts > tmax) tmax = ts;
    pbase += (int64_t)s.cam.width * s.cam.height;
  }
  // one session travels in the launch arguments (Batch::one); the table is
  // uploaded for several, and for the raster variants that read it whatever
  // the count (saved fragments, lanes by previous work)
  const bool table = ns > 1 ||
                     (fwd ? (flags & (RTGS_FWD_SAVE_FRAGMENTS | RTGS_FWD_BALANCE_LANES)) != 0
                          : (flags & (RTGS_GRAD_SAVED_FRAGMENTS | RTGS_GRAD_BALANCED_LANES)) != 0);
  if (table) {
    e = hipMemcpyAsync(w.table, t, sizeof(SessionDev) * ns, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(session table)");
  }
  B.one = t[0];
  e = hipEventRecord(h->ring_ev[slot], st);
  if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
  B.sess = w.table;
  B.n_sessions = ns;
  B.n_total = gbase;
  B.t_total = tbase;
  B.b_total = bbase;
  B.c_total = cbase;
  B.t_max = tmax;
  return RTGS_OK;
}

int32_t prepare(rtgs_handle_t h, const rtgs_session* ss, int32_t ns, void* ws, uint64_t ws_bytes,
                int64_t cap, WsLayout& L, WsPtrs& w, bool frags = false) {
  if (!h) return fail(RTGS_ERR_INVALID_ARG, "null handle");
  if (!ss) return fail(RTGS_ERR_INVALID_ARG, "null sessions");
  if (ns < 1 || ns > RTGS_MAX_SESSIONS)
    return fail(RTGS_ERR_INVALID_ARG, "n_sessions %d outside [1, %d]", ns, RTGS_MAX_SESSIONS);
  int32_t r = check_cap(cap);
  if (r) return r;
  std::vector<int32_t> n(ns), wd(ns), ht(ns), js(ns);
  for (int i = 0; i < ns; ++i) {
    n[i] = ss[i].g.n;
    wd[i] = ss[i].cam.width;
    ht[i] = ss[i].cam.height;
    js[i] = ss[i].sample_log2;
    if (js[i] > 0 && !ss[i].pixel_mask)
      return fail(RTGS_ERR_INVALID_ARG, "session %d: sample_log2 > 0 needs a pixel mask", i);
  }
  Counts g;
  r = geometry(n.data(), wd.data(), ht.data(), ns, g, js.data());
  if (r) return r;
  if (!ws) return fail(RTGS_ERR_INVALID_ARG, "null workspace");
  L = make_layout(g, cap, frags);
  if (ws_bytes < L.total)
    return fail(RTGS_ERR_WORKSPACE, "workspace %llu bytes < required %llu",
                (unsigned long long)ws_bytes, (unsigned long long)L.total);
  if (reinterpret_cast<uintptr_t>(ws) % kAlign)
    return fail(RTGS_ERR_INVALID_ARG, "workspace not 256-byte aligned");
  w = ws_ptrs(ws, L);
  return RTGS_OK;
}

rtgs_session single(const rtgs_gaussians* g, const rtgs_camera* cam, const uint8_t* pmask) {
  rtgs_session s{};
  s.g = *g;
  s.cam = *cam;
  s.pixel_mask = pmask;
  return s;
}

}  // namespace

extern "C" {

const char* rtgs_last_error(void) { return g_err.c_str(); }

int32_t rtgs_create(rtgs_handle_t* out, int32_t device) {
  if (!out) return fail(RTGS_ERR_INVALID_ARG, "null output handle");
  *out = nullptr;
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
  if (device < 0 || device >= count)
    return fail(RTGS_ERR_INVALID_ARG, "device %d outside [0, %d)", device, count);
  e = hipSetDevice(device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  auto* h = new rtgs_context();
  h->device = device;
  e = hipMalloc(&h->d_scalars, 64);
  if (e == hipSuccess) e = hipMemset(h->d_scalars, 0, 64);
  if (e == hipSuccess) e = hipMalloc(&h->d_prune, sizeof(uint32_t) * kPruneScratchWords);
  if (e == hipSuccess)
    e = hipHostMalloc(&h->h_ring, sizeof(SessionDev) * RTGS_MAX_SESSIONS * kRing,
                      hipHostMallocDefault);
  for (int i = 0; i < kRing && e == hipSuccess; ++i)
    e = hipEventCreateWithFlags(&h->ring_ev[i], hipEventDisableTiming);
  if (e != hipSuccess) {
    rtgs_destroy(h);
    return hip_fail(e, "rtgs_create");
  }
  *out = h;
  return RTGS_OK;
}

int32_t rtgs_destroy(rtgs_handle_t h) {
  if (!h) return RTGS_OK;
  (void)hipDeviceSynchronize();
  for (int i = 0; i < kRing; ++i)
    if (h->ring_ev[i]) (void)hipEventDestroy(h->ring_ev[i]);
  if (h->h_ring) (void)hipHostFree(h->h_ring);
  if (h->d_prune) (void)hipFree(h->d_prune);
  if (h->d_scalars) (void)hipFree(h->d_scalars);
  delete h;
  return RTGS_OK;
}

int32_t rtgs_workspace_size_batched(const int32_t* n, const int32_t* width, const int32_t* height,
                                    int32_t n_sessions, int64_t pair_capacity, int32_t flags,
                                    uint64_t* bytes) {
  if (!n || !width || !height || !bytes) return fail(RTGS_ERR_INVALID_ARG, "null argument");
  int32_t r = check_cap(pair_capacity);
  if (r) return r;
  Counts g;
  r = geometry(n, width, height, n_sessions, g);
  if (r) return r;
  *bytes = make_layout(g, pair_capacity, (flags & RTGS_FWD_SAVE_FRAGMENTS) != 0).total;
  return RTGS_OK;
}

int32_t rtgs_workspace_size(int32_t n, int32_t width, int32_t height, int64_t pair_capacity,
                            int32_t flags, uint64_t* bytes) {
  if (!bytes) return fail(RTGS_ERR_INVALID_ARG, "null argument");
  int32_t r = check_cap(pair_capacity);
  if (r) return r;
  const int32_t j = (flags >> RTGS_SAMPLE_SHIFT) & 0xf;
  Counts g;
  r = geometry(&n, &width, &height, 1, g, &j);
  if (r) return r;
  *bytes = make_layout(g, pair_capacity, (flags & RTGS_FWD_SAVE_FRAGMENTS) != 0).total;
  return RTGS_OK;
}

int32_t render_fwd_batched(rtgs_handle_t h, const rtgs_session* ss, int32_t ns, void* ws,
                           uint64_t ws_bytes, int64_t cap, int32_t flags, void* stream) {
  if (flags & ~(RTGS_FWD_SAVE_STATE | RTGS_FWD_STATS | RTGS_FWD_REUSE_LISTS |
                RTGS_FWD_SAVE_FRAGMENTS | RTGS_FWD_BALANCE_LANES))
    return fail(RTGS_ERR_INVALID_ARG, "unknown flags %d (sample_log2 goes in the sessions)",
                flags);
  const bool frags = (flags & RTGS_FWD_SAVE_FRAGMENTS) != 0;
  if (frags && !(flags & RTGS_FWD_SAVE_STATE))
    return fail(RTGS_ERR_INVALID_ARG, "RTGS_FWD_SAVE_FRAGMENTS needs RTGS_FWD_SAVE_STATE");
  WsLayout L;
  WsPtrs w;
  int32_t r = prepare(h, ss, ns, ws, ws_bytes, cap, L, w, frags);
  if (r) return r;
  for (int i = 0; i < ns; ++i) {
    if ((r = check_session(ss[i], i, true, flags))) return r;
    if ((flags & RTGS_FWD_STATS) && !ss[i].stats)
      return fail(RTGS_ERR_INVALID_ARG, "session %d: RTGS_FWD_STATS needs stats", i);
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  Batch B;
  r = upload_table(h, ss, ns, w, st, true, flags, B);
  if (r) return r;
  StageTimer* tm = h->timer.mask ? &h->timer : nullptr;
  hipError_t e = launch_forward_prep(B, w, h->d_scalars, (flags & RTGS_FWD_REUSE_LISTS) != 0,
                                     st, tm);
  if (e == hipSuccess)
    e = launch_raster_fwd(B, w, (flags & RTGS_FWD_STATS) != 0, frags,
                          (flags & RTGS_FWD_BALANCE_LANES) != 0, st, tm);
  if (e != hipSuccess) return hip_fail(e, "render_fwd launch");
  h->last_stream = st;
  h->used = true;
  return RTGS_OK;
}

int32_t render_bwd_batched(rtgs_handle_t h, const rtgs_session* ss, int32_t ns, void* ws,
                           uint64_t ws_bytes, int64_t cap, int32_t flags, void* stream) {
  const int32_t known = RTGS_GRAD_POSE | RTGS_GRAD_MAP | RTGS_GRAD_COV3D |
                        RTGS_GRAD_RECOMPUTE_STATE | RTGS_GRAD_SCORE | RTGS_GRAD_SAVED_FRAGMENTS |
                        RTGS_GRAD_BALANCED_LANES | RTGS_GRAD_ADAM;
  if (flags & ~known) return fail(RTGS_ERR_INVALID_ARG, "unknown flags %d", flags);
  if ((flags & RTGS_GRAD_ADAM) && !(flags & RTGS_GRAD_MAP))
    return fail(RTGS_ERR_INVALID_ARG, "RTGS_GRAD_ADAM needs RTGS_GRAD_MAP");
  if (!(flags & (RTGS_GRAD_POSE | RTGS_GRAD_MAP | RTGS_GRAD_SCORE)))
    return fail(RTGS_ERR_INVALID_ARG, "render_bwd needs RTGS_GRAD_POSE, MAP or SCORE");
  const bool frags = (flags & RTGS_GRAD_SAVED_FRAGMENTS) != 0;
  if (frags && (flags & RTGS_GRAD_RECOMPUTE_STATE))
    return fail(RTGS_ERR_INVALID_ARG, "saved fragments come with saved state, not recompute");
  const bool bal = (flags & RTGS_GRAD_BALANCED_LANES) != 0;
  if (bal && (flags & RTGS_GRAD_RECOMPUTE_STATE))
    return fail(RTGS_ERR_INVALID_ARG, "balanced lanes come with saved state, not recompute");
  WsLayout L;
  WsPtrs w;
  int32_t r = prepare(h, ss, ns, ws, ws_bytes, cap, L, w, frags);
  if (r) return r;
  for (int i = 0; i < ns; ++i)
    if ((r = check_session(ss[i], i, false, flags))) return r;
  hipStream_t st = static_cast<hipStream_t>(stream);
  Batch B;
  r = upload_table(h, ss, ns, w, st, false, flags, B);
  if (r) return r;
  StageTimer* tm = h->timer.mask ? &h->timer : nullptr;
  hipError_t e = hipSuccess;
  if (flags & RTGS_GRAD_RECOMPUTE_STATE) e = launch_raster_fwd(B, w, false, false, false, st, tm);
  bool alpha_grad = false;            // some session passes dL/dA
  for (int i = 0; i < ns; ++i) alpha_grad = alpha_grad || ss[i].dL_dalpha != nullptr;
  if (e == hipSuccess)
    e = launch_raster_bwd(B, w, (flags & RTGS_GRAD_MAP) ? 0 : 1, alpha_grad, frags, bal, st,
                          tm);
  if (e == hipSuccess) e = launch_preprocess_bwd(B, w, flags, st, tm);
  if (e != hipSuccess) return hip_fail(e, "render_bwd launch");
  h->last_stream = st;
  h->used = true;
  return RTGS_OK;
}

int32_t render_fwd(rtgs_handle_t h, const rtgs_gaussians* g, const rtgs_camera* cam,
                   const uint8_t* pixel_mask, void* ws, uint64_t ws_bytes, int64_t cap,
                   float* out_color, float* out_depth, float* out_alpha, float* final_T,
                   int32_t* last_idx, uint8_t* visible_out, int32_t flags, void* stream) {
  if (!g || !cam) return fail(RTGS_ERR_INVALID_ARG, "null gaussians or camera");
  rtgs_session s = single(g, cam, pixel_mask);
  s.sample_log2 = (flags >> RTGS_SAMPLE_SHIFT) & 0xf;
  flags &= ~(0xf << RTGS_SAMPLE_SHIFT);
  s.color = out_color;
  s.depth = out_depth;
  s.alpha = out_alpha;
  s.final_T = final_T;
  s.last_idx = last_idx;
  s.visible = visible_out;
  return render_fwd_batched(h, &s, 1, ws, ws_bytes, cap, flags, stream);
}

int32_t render_bwd(rtgs_handle_t h, const rtgs_gaussians* g, const rtgs_camera* cam,
                   const uint8_t* pixel_mask, void* ws, uint64_t ws_bytes, int64_t cap,
                   const float* final_T, const int32_t* last_idx, const float* dL_dcolor,
                   const float* dL_ddepth, const float* dL_dalpha, int32_t grad_flags,
                   float* g_means, float* g_log_scales, float* g_quats, float* g_opacity_logits,
                   float* g_colors, float* g_pose6, float* g_viewmat, float* g_cov3d,
                   void* stream) {
  if (!g || !cam) return fail(RTGS_ERR_INVALID_ARG, "null gaussians or camera");
  if (grad_flags & RTGS_GRAD_ADAM)
    return fail(RTGS_ERR_INVALID_ARG, "RTGS_GRAD_ADAM takes render_bwd_batched (its Adam state)");
  rtgs_session s = single(g, cam, pixel_mask);
  s.sample_log2 = (grad_flags >> RTGS_SAMPLE_SHIFT) & 0xf;
  grad_flags &= ~(0xf << RTGS_SAMPLE_SHIFT);
  s.final_T = const_cast<float*>(final_T);
  s.last_idx = const_cast<int32_t*>(last_idx);
  s.dL_dcolor = dL_dcolor;
  s.dL_ddepth = dL_ddepth;
  s.dL_dalpha = dL_dalpha;
  s.g_means = g_means;
  s.g_log_scales = g_log_scales;
  s.g_quats = g_quats;
  s.g_opacity_logits = g_opacity_logits;
  s.g_colors = g_colors;
  s.g_pose6 = g_pose6;
  s.g_viewmat = g_viewmat;
  s.g_cov3d = g_cov3d;
  return render_bwd_batched(h, &s, 1, ws, ws_bytes, cap, grad_flags, stream);
}

int32_t prune_by_grad(rtgs_handle_t h, const float* g_means, const float* g_cov3d,
                      const uint8_t* visible, const uint8_t* mask_in, int32_t n, float lambda,
                      float max_ratio, uint8_t* mask_out, int32_t* n_masked_dev,
                      float* score_out, void* stream) {
  if (!h) return fail(RTGS_ERR_INVALID_ARG, "null handle");
  if (n < 0) return fail(RTGS_ERR_INVALID_ARG, "n = %d < 0", n);
  if (n > 0 && (!g_means || !g_cov3d || !mask_out))
    return fail(RTGS_ERR_INVALID_ARG, "null gradient or mask_out");
  if (!(max_ratio >= 0.f && max_ratio <= 0.5f))
    return fail(RTGS_ERR_INVALID_ARG, "max_ratio %g outside [0, 0.5]", (double)max_ratio);
  if (!std::isfinite(lambda) || lambda < 0.f)
    return fail(RTGS_ERR_INVALID_ARG, "lambda %g must be finite and >= 0", (double)lambda);
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = launch_prune(g_means, g_cov3d, visible, mask_in, n, lambda, max_ratio, mask_out,
                              n_masked_dev, score_out, h->d_prune, st);
  if (e != hipSuccess) return hip_fail(e, "prune_by_grad launch");
  return RTGS_OK;
}

int32_t downsample_mask(const float* final_T, int32_t width, int32_t height, int32_t log2_ratio,
                        uint8_t* mask_out, int32_t* n_active_dev, void* stream) {
  if (!final_T || !mask_out) return fail(RTGS_ERR_INVALID_ARG, "null final_T or mask_out");
  if (width <= 0 || height <= 0)
    return fail(RTGS_ERR_INVALID_ARG, "image %d x %d", width, height);
  if (log2_ratio < 0 || log2_ratio > 8)
    return fail(RTGS_ERR_INVALID_ARG, "log2_ratio %d outside [0, 8]", log2_ratio);
  hipError_t e = launch_downsample(final_T, width, height, log2_ratio, mask_out, n_active_dev,
                                   static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "downsample_mask launch");
  return RTGS_OK;
}

int32_t adam_step(rtgs_handle_t h, const rtgs_adam_group* groups, int32_t n_groups, double beta1,
                  double beta2, double eps, void* stream) {
  if (!h) return fail(RTGS_ERR_INVALID_ARG, "null handle");
  if (n_groups < 0 || (n_groups > 0 && !groups))
    return fail(RTGS_ERR_INVALID_ARG, "bad group list (n_groups = %d)", n_groups);
  if (!(beta1 >= 0.0 && beta1 < 1.0 && beta2 >= 0.0 && beta2 < 1.0))
    return fail(RTGS_ERR_INVALID_ARG, "betas (%g, %g) outside [0, 1)", beta1, beta2);
  if (!(eps >= 0.0) || !std::isfinite(eps))
    return fail(RTGS_ERR_INVALID_ARG, "eps %g must be finite and >= 0", eps);
  for (int i = 0; i < n_groups; ++i) {
    const rtgs_adam_group& g = groups[i];
    if (g.n < 0) return fail(RTGS_ERR_INVALID_ARG, "group %d: n = %lld < 0", i, (long long)g.n);
    if (g.n > 0 && (!g.param || !g.grad || !g.exp_avg || !g.exp_avg_sq))
      return fail(RTGS_ERR_INVALID_ARG, "group %d: null array", i);
    if (g.step < 1) return fail(RTGS_ERR_INVALID_ARG, "group %d: step %d < 1", i, g.step);
    if (!std::isfinite(g.lr)) return fail(RTGS_ERR_INVALID_ARG, "group %d: lr not finite", i);
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  StageTimer* tm = h->timer.mask ? &h->timer : nullptr;
  const int64_t per_block = 256 * kAdamPerThread;
  for (int first = 0; first < n_groups; first += kAdamMaxGroups) {
    AdamArgs a{};
    // 1 - beta is formed in double: float32(beta2 = 0.999) alone would
    // carry a 1e-5 relative error into 1 - beta2
    a.beta1 = (float)beta1;
    a.beta2 = (float)beta2;
    a.omb1 = (float)(1.0 - beta1);
    a.omb2 = (float)(1.0 - beta2);
    a.eps = (float)eps;
    int64_t blocks = 0;
    for (int i = first; i < n_groups && i < first + kAdamMaxGroups; ++i) {
      const rtgs_adam_group& g = groups[i];
      if (g.n == 0) continue;
      AdamGroupDev& d = a.grp[a.n_groups++];
      d.p = g.param;
      d.g = g.grad;
      d.m = g.exp_avg;
      d.v = g.exp_avg_sq;
      d.n = g.n;
      const double bc1 = 1.0 - std::pow(beta1, (double)g.step);
      const double bc2 = 1.0 - std::pow(beta2, (double)g.step);
      d.step_size = (float)((double)g.lr / bc1);
      d.inv_sqrt_bc2 = (float)(1.0 / std::sqrt(bc2));
      auto al = [](const void* q) { return (reinterpret_cast<uintptr_t>(q) & 15u) == 0; };
      d.vec = al(g.param) && al(g.grad) && al(g.exp_avg) && al(g.exp_avg_sq);
      d.block0 = (int32_t)blocks;
      blocks += (g.n + per_block - 1) / per_block;
      if (blocks > (int64_t)INT32_MAX) return fail(RTGS_ERR_INVALID_ARG, "too many elements");
    }
    a.n_blocks = (int32_t)blocks;
    hipError_t e = launch_adam(a, st, tm);
    if (e != hipSuccess) return hip_fail(e, "adam_step launch");
  }
  return RTGS_OK;
}

int32_t loss_l1_grad(const float* color, const float* depth, const float* target_color,
                     const float* target_depth, const uint8_t* pixel_mask,
                     const int32_t* n_active_dev, int32_t width, int32_t height,
                     float w_color, float w_depth, float* dL_dcolor, float* dL_ddepth,
                     void* stream) {
  if (width <= 0 || height <= 0)
    return fail(RTGS_ERR_INVALID_ARG, "image %d x %d", width, height);
  if (!color || !depth || !target_color || !target_depth || !dL_dcolor || !dL_ddepth)
    return fail(RTGS_ERR_INVALID_ARG, "null image or gradient");
  if (pixel_mask && !n_active_dev)
    return fail(RTGS_ERR_INVALID_ARG, "a pixel mask needs its active-pixel count");
  if (!std::isfinite(w_color) || !std::isfinite(w_depth))
    return fail(RTGS_ERR_INVALID_ARG, "weights must be finite");
  LossArgs a{color, depth, target_color, target_depth, pixel_mask, n_active_dev,
             dL_dcolor, dL_ddepth, width, height, w_color, w_depth};
  hipError_t e = launch_l1_grad(a, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "loss_l1_grad launch");
  return RTGS_OK;
}

int32_t loss_l1_grad_batched(const rtgs_loss_item* items, int32_t n_items, float w_color,
                             float w_depth, void* stream) {
  if (n_items < 0 || (n_items > 0 && !items))
    return fail(RTGS_ERR_INVALID_ARG, "bad item list (n_items = %d)", n_items);
  if (!std::isfinite(w_color) || !std::isfinite(w_depth))
    return fail(RTGS_ERR_INVALID_ARG, "weights must be finite");
  for (int i = 0; i < n_items; ++i) {
    const rtgs_loss_item& it = items[i];
    if (it.width <= 0 || it.height <= 0)
      return fail(RTGS_ERR_INVALID_ARG, "item %d: image %d x %d", i, it.width, it.height);
    if (!it.color || !it.depth || !it.target_color || !it.target_depth || !it.dL_dcolor ||
        !it.dL_ddepth)
      return fail(RTGS_ERR_INVALID_ARG, "item %d: null image or gradient", i);
    if (it.pixel_mask && !it.n_active_dev)
      return fail(RTGS_ERR_INVALID_ARG, "item %d: a pixel mask needs its active-pixel count", i);
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  for (int first = 0; first < n_items; first += kLossMaxItems) {
    LossBatchArgs a{};
    int blocks = 0;
    for (int i = first; i < n_items && i < first + kLossMaxItems; ++i) {
      const rtgs_loss_item& it = items[i];
      LossItemDev& d = a.item[a.n++];
      d.a = LossArgs{it.color, it.depth, it.target_color, it.target_depth, it.pixel_mask,
                     it.n_active_dev, it.dL_dcolor, it.dL_ddepth, it.width, it.height,
                     w_color, w_depth};
      d.block_base = blocks;
      blocks += (int)(((int64_t)it.width * it.height + 255) / 256);
    }
    hipError_t e = launch_l1_grad_batched(a, blocks, st);
    if (e != hipSuccess) return hip_fail(e, "loss_l1_grad_batched launch");
  }
  return RTGS_OK;
}

int32_t pose_update(const rtgs_pose_item* items, int32_t n, double beta1, double beta2,
                    double eps, void* stream) {
  if (n < 0 || (n > 0 && !items)) return fail(RTGS_ERR_INVALID_ARG, "bad item list (n = %d)", n);
  if (!(beta1 >= 0.0 && beta1 < 1.0 && beta2 >= 0.0 && beta2 < 1.0))
    return fail(RTGS_ERR_INVALID_ARG, "betas (%g, %g) outside [0, 1)", beta1, beta2);
  if (!(eps >= 0.0) || !std::isfinite(eps))
    return fail(RTGS_ERR_INVALID_ARG, "eps %g must be finite and >= 0", eps);
  for (int i = 0; i < n; ++i) {
    const rtgs_pose_item& it = items[i];
    if (!it.viewmat || !it.g_pose6 || !it.exp_avg || !it.exp_avg_sq)
      return fail(RTGS_ERR_INVALID_ARG, "item %d: null array", i);
    if (it.step < 1) return fail(RTGS_ERR_INVALID_ARG, "item %d: step %d < 1", i, it.step);
    if (!std::isfinite(it.lr_rho) || !std::isfinite(it.lr_phi))
      return fail(RTGS_ERR_INVALID_ARG, "item %d: learning rate not finite", i);
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  for (int first = 0; first < n; first += kPoseMaxItems) {
    PoseArgs a{};
    a.beta1 = beta1;
    a.beta2 = beta2;
    a.eps = eps;
    for (int i = first; i < n && i < first + kPoseMaxItems; ++i) {
      const rtgs_pose_item& it = items[i];
      PoseItemDev& d = a.item[a.n++];
      d.viewmat = it.viewmat;
      d.g_pose6 = it.g_pose6;
      d.exp_avg = it.exp_avg;
      d.exp_avg_sq = it.exp_avg_sq;
      d.lr_rho = it.lr_rho;
      d.lr_phi = it.lr_phi;
      d.bc1 = 1.0 - std::pow(beta1, (double)it.step);
      d.bc2 = 1.0 - std::pow(beta2, (double)it.step);
    }
    hipError_t e = launch_pose_update(a, st);
    if (e != hipSuccess) return hip_fail(e, "pose_update launch");
  }
  return RTGS_OK;
}

uint64_t rtgs_compact_scratch_size(int32_t n) {
  const uint64_t nb = n > 0 ? ((uint64_t)n + kCompactBlock - 1) / kCompactBlock : 0;
  return 4 * (nb + 1);
}

// Validates a compaction call and fills its kernel arguments (scratch not set).
static int32_t compact_args(const uint8_t* drop, int32_t n, const rtgs_compact_item* items,
                            int32_t n_items, int32_t* n_kept, CompactArgs& a) {
  if (n < 0) return fail(RTGS_ERR_INVALID_ARG, "n = %d", n);
  if (n_items < 0 || n_items > kCompactMaxItems || (n_items > 0 && !items))
    return fail(RTGS_ERR_INVALID_ARG, "bad item list (n_items = %d)", n_items);
  if (!n_kept || (n > 0 && !drop))
    return fail(RTGS_ERR_INVALID_ARG, "null drop mask or count");
  for (int i = 0; i < n_items; ++i) {
    const rtgs_compact_item& it = items[i];
    if ((n > 0 && !it.src) || (it.dst_rows > 0 && !it.dst) || it.row_bytes <= 0 ||
        it.dst_rows < 0)
      return fail(RTGS_ERR_INVALID_ARG, "item %d: null array, row_bytes %d or dst_rows %d", i,
                  it.row_bytes, it.dst_rows);
    const uint64_t sb = (uint64_t)n * (uint64_t)it.row_bytes;
    const uint64_t db = (uint64_t)it.dst_rows * (uint64_t)it.row_bytes;
    const uintptr_t s0 = (uintptr_t)it.src, d0 = (uintptr_t)it.dst;
    if (sb > 0 && db > 0 && s0 < d0 + db && d0 < s0 + sb)
      return fail(RTGS_ERR_INVALID_ARG, "item %d: dst overlaps src", i);
    if (it.row_bytes % 4 == 0 && ((s0 | d0) & 3u))
      return fail(RTGS_ERR_INVALID_ARG, "item %d: rows of %d bytes need 4-byte alignment", i,
                  it.row_bytes);
    a.item[i].src = static_cast<const unsigned char*>(it.src);
    a.item[i].dst = static_cast<unsigned char*>(it.dst);
    a.item[i].row_bytes = it.row_bytes;
    a.item[i].dst_rows = it.dst_rows;
  }
  a.n_items = n_items;
  a.n = n;
  a.drop = drop;
  a.n_kept = n_kept;
  return RTGS_OK;
}

int32_t compact_by_mask(const uint8_t* drop, int32_t n, const rtgs_compact_item* items,
                        int32_t n_items, void* scratch, uint64_t scratch_bytes, int32_t* n_kept,
                        void* stream) {
  CompactArgs a{};
  int32_t r = compact_args(drop, n, items, n_items, n_kept, a);
  if (r) return r;
  if (!scratch) return fail(RTGS_ERR_INVALID_ARG, "null scratch");
  if (scratch_bytes < rtgs_compact_scratch_size(n))
    return fail(RTGS_ERR_WORKSPACE, "compaction scratch %llu < %llu bytes",
                (unsigned long long)scratch_bytes,
                (unsigned long long)rtgs_compact_scratch_size(n));
  a.block_keep = static_cast<uint32_t*>(scratch);
  hipError_t e = launch_compact(a, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "compact_by_mask launch");
  return RTGS_OK;
}

int32_t compact_by_mask_static(const uint8_t* drop, int32_t n, const rtgs_compact_item* items,
                               int32_t n_items, int32_t* n_kept, void* stream) {
  CompactArgs a{};
  int32_t r = compact_args(drop, n, items, n_items, n_kept, a);
  if (r) return r;
  if (n > RTGS_COMPACT_STATIC_MAX_ROWS)
    return fail(RTGS_ERR_WORKSPACE,
                "compact_by_mask_static: n = %d rows exceeds the static scratch's maximum of "
                "%d rows (use compact_by_mask with a caller scratch)",
                n, RTGS_COMPACT_STATIC_MAX_ROWS);
  static_assert(RTGS_COMPACT_STATIC_MAX_ROWS ==
                    (int64_t)(kCompactStaticWords - 1) * kCompactBlock,
                "the header's row limit matches the device scratch");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (st) {
    int cur = 0, sd = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e == hipSuccess) e = hipStreamGetDevice(st, &sd);
    if (e != hipSuccess) return hip_fail(e, "compact_by_mask_static device query");
    if (sd != cur)
      return fail(RTGS_ERR_INVALID_ARG,
                  "compact_by_mask_static: the stream belongs to device %d, device %d is current",
                  sd, cur);
  }
  uint32_t* ptr = nullptr;
  hipError_t e = compact_static_scratch(&ptr);
  if (e != hipSuccess) return hip_fail(e, "compact_by_mask_static scratch address");
  a.block_keep = ptr;
  e = launch_compact(a, st);
  if (e != hipSuccess) return hip_fail(e, "compact_by_mask_static launch");
  return RTGS_OK;
}

int32_t rtgs_tile_rects(int32_t n, int32_t width, int32_t height, int32_t sample_log2,
                        int64_t pair_capacity, const void* ws, uint64_t ws_bytes,
                        int32_t* rect_out, void* stream) {
  if (!ws || (n > 0 && !rect_out)) return fail(RTGS_ERR_INVALID_ARG, "null argument");
  int32_t r = check_cap(pair_capacity);
  if (r) return r;
  Counts g;
  r = geometry(&n, &width, &height, 1, g, &sample_log2);
  if (r) return r;
  const WsLayout L = make_layout(g, pair_capacity);
  if (ws_bytes < L.total) return fail(RTGS_ERR_WORKSPACE, "workspace too small");
  if (n == 0) return RTGS_OK;
  const WsPtrs w = ws_ptrs(const_cast<void*>(ws), L);
  Batch B{};
  B.n_total = (int32_t)g.n_total;
  B.t_total = (int32_t)g.t_total;
  hipError_t e = launch_debug_stage(B, w, nullptr, rect_out, nullptr, nullptr, 0,
                                    static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "rtgs_tile_rects launch");
  return RTGS_OK;
}

int32_t tile_pair_change(const int32_t* rect_ref, const int32_t* rect_cur, const uint8_t* skip,
                         int32_t n, int64_t* out, void* stream) {
  if (n < 0 || !out || (n > 0 && (!rect_ref || !rect_cur)))
    return fail(RTGS_ERR_INVALID_ARG, "bad arguments (n = %d)", n);
  hipError_t e = launch_rect_change(rect_ref, rect_cur, skip, n, out,
                                    static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "tile_pair_change launch");
  return RTGS_OK;
}

int32_t rtgs_downsample_log2_ratio(int32_t is_keyframe, int32_t n, int32_t k, int32_t m) {
  if (is_keyframe) return 0;
  if (n <= k || m < 2)
    return fail(RTGS_ERR_INVALID_ARG, "non-keyframe needs n > k and m >= 2");
  const double steps = (double)(n - k - 1) * std::log2((double)m);
  const int j = 4 - (int)std::floor(steps + 1e-12);
  return j < 2 ? 2 : j;
}

int32_t rtgs_query(rtgs_handle_t h, int32_t blocking, int64_t* pairs_needed, int32_t* state) {
  if (!h) return fail(RTGS_ERR_INVALID_ARG, "null handle");
  if (state) *state = RTGS_STATE_IDLE;
  if (!h->used) {
    if (pairs_needed) *pairs_needed = 0;
    return RTGS_OK;
  }
  hipStream_t st = h->last_stream;
  if (!blocking) {
    hipError_t q = hipStreamQuery(st);
    if (q == hipErrorNotReady) {
      if (state) *state = RTGS_STATE_EXECUTING;
      return RTGS_OK;
    }
    if (q != hipSuccess) return hip_fail(q, "hipStreamQuery");
  }
  unsigned long long got[2] = {0, 0}, zero[2] = {0, 0};
  hipError_t e = hipMemcpyAsync(got, h->d_scalars, sizeof(got), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(h->d_scalars, zero, sizeof(zero), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "rtgs_query");
  if (got[1] > 0) {
    if (pairs_needed) *pairs_needed = (int64_t)got[1];
    return fail(RTGS_ERR_CAPACITY, "a render needed %llu pairs, more than its capacity",
                (unsigned long long)got[1]);
  }
  if (pairs_needed) *pairs_needed = (int64_t)got[0];
  return RTGS_OK;
}

int32_t rtgs_debug_stage(const int32_t* n, const int32_t* width, const int32_t* height,
                         const int32_t* sample_log2, int32_t n_sessions, int64_t pair_capacity,
                         const void* ws, uint64_t ws_bytes, float* stage, int32_t* rect,
                         int32_t* ranges, int32_t* ids, int64_t ids_capacity, void* stream) {
  if (!n || !width || !height || !ws) return fail(RTGS_ERR_INVALID_ARG, "null argument");
  int32_t r = check_cap(pair_capacity);
  if (r) return r;
  Counts g;
  r = geometry(n, width, height, n_sessions, g, sample_log2);
  if (r) return r;
  const WsLayout L = make_layout(g, pair_capacity);
  if (ws_bytes < L.total) return fail(RTGS_ERR_WORKSPACE, "workspace too small");
  const WsPtrs w = ws_ptrs(const_cast<void*>(ws), L);
  Batch B{};
  B.n_total = (int32_t)g.n_total;
  B.t_total = (int32_t)g.t_total;
  hipError_t e = launch_debug_stage(B, w, stage, rect, ranges, ids, ids_capacity,
                                    static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "rtgs_debug_stage launch");
  return RTGS_OK;
}

int32_t rtgs_profile_enable(rtgs_handle_t h, int32_t stage_mask) {
  if (!h) return fail(RTGS_ERR_INVALID_ARG, "null handle");
  h->timer.mask = stage_mask & ((1 << RTGS_PROFILE_STAGES) - 1);
  return RTGS_OK;
}

int32_t rtgs_profile_read(rtgs_handle_t h, double* total_ms, int64_t* launches) {
  if (!h || !total_ms || !launches) return fail(RTGS_ERR_INVALID_ARG, "null argument");
  for (int i = 0; i < RTGS_PROFILE_STAGES; ++i) {
    total_ms[i] = 0.0;
    launches[i] = 0;
  }
  EventTimer& t = h->timer;
  hipError_t e = t.err;
  t.err = hipSuccess;
  for (auto& r : t.recs) {
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventSynchronize(r.b);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.a, r.b);
    if (e == hipSuccess && r.stage < RTGS_PROFILE_STAGES) {
      total_ms[r.stage] += ms;
      launches[r.stage] += 1;
    }
    t.pool.push_back(r.a);
    t.pool.push_back(r.b);
  }
  t.recs.clear();
  if (e != hipSuccess) return hip_fail(e, "rtgs_profile_read");
  return RTGS_OK;
}

int32_t rtgs_selftest_wave_sum(const float* in, float* out, int32_t n_waves, void* stream) {
  if (n_waves < 0 || (n_waves > 0 && (!in || !out)))
    return fail(RTGS_ERR_INVALID_ARG, "bad arguments");
  hipError_t e = launch_wave_sum_test(in, out, n_waves, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "wave sum launch");
  return RTGS_OK;
}

}  // extern "C"
