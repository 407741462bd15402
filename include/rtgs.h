/*
 * rtgs.h - C ABI of librtgs, the MI355X (gfx950) differentiable tile-based
 * Gaussian-splatting rasterizer used by 3DGS-SLAM tracking and mapping.
 *
 * The operations follow the paper's rendering pipeline (Sec. 2.1, Steps 1-3)
 * and its backpropagation (Sec. 2.2, Steps 4-5), plus the two redundancy
 * reductions of Sec. 4 (adaptive Gaussian pruning, dynamic downsampling).
 * The status query mirrors the paper's programming model (Sec. 5.5).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every function returns an int32 status (RTGS_OK or a negative RTGS_ERR_*)
 *   and never throws.  rtgs_last_error() returns a message for the calling
 *   thread's last failure.
 * - All array arguments are DEVICE pointers unless stated otherwise; they are
 *   owned by the caller, must stay alive until the work on `stream` has
 *   finished, and are never freed by the library.  Inputs are read-only;
 *   outputs are overwritten, never accumulated.
 * - `stream` is a hipStream_t passed as void*; every call only enqueues work
 *   on it (asynchronous).  NULL means the default stream.
 * - Layouts are contiguous float32:
 *     means [n][3], log_scales [n][3] (log standard deviations per axis),
 *     quats [n][4] as (w, x, y, z) (normalised inside), opacity_logits [n],
 *     colors [n][3] (RGB, spherical harmonics of degree 0);
 *     images are planar: color [3][H][W], depth/alpha/final_T [H][W];
 *     viewmat is a device array of 12 floats, row-major 3x4 world->camera.
 *   Pixel (i, j) samples the image plane at (i + 0.5, j + 0.5); depth is the
 *   camera-space z.
 * - A handle (rtgs_create) owns only small host/device scalars, an event and
 *   a ring of pinned staging buffers; use one handle per stream.
 * - Workspace: the caller allocates `ws` of the size given by
 *   rtgs_workspace_size*, and passes the same `ws` to render_fwd and to the
 *   render_bwd that follows it (the backward reuses the forward's projected
 *   Gaussians, tile lists and depth order, and each list entry's quadrant
 *   mask: the sort is not redone, Sec. 2.2); no other render_fwd may use
 *   that workspace in between.
 * - Pair capacity: the number of (tile, Gaussian) pairs is data dependent.
 *   The caller sizes the pair buffer (`pair_capacity`); if a frame needs more,
 *   the excess pairs are dropped on the device (no fault), the output of that
 *   call is invalid, and rtgs_query() reports RTGS_ERR_CAPACITY together
 *   with the number of pairs needed.  Nothing forces a host sync.
 */
#ifndef RTGS_H
#define RTGS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---- */
#define RTGS_OK               0
#define RTGS_ERR_INVALID_ARG (-1)  /* null pointer, n < 0, W/H <= 0, bad flag  */
#define RTGS_ERR_CAPACITY    (-2)  /* pair buffer too small (see rtgs_query)  */
#define RTGS_ERR_HIP         (-3)  /* a HIP runtime call failed                */
#define RTGS_ERR_WORKSPACE   (-4)  /* workspace smaller than required          */

/* ---- render_fwd flags ---- */
#define RTGS_FWD_SAVE_STATE   1   /* write final_T and last_idx (saved state)  */
#define RTGS_FWD_REUSE_LISTS  4   /* keep the tile lists of this workspace's
                                     last forward (see render_fwd)            */
#define RTGS_FWD_STATS        2   /* write per-pixel work counts (sessions'
                                     `stats`; render_fwd_batched only)         */
#define RTGS_FWD_SAVE_FRAGMENTS 16 /* also save every blended fragment's
                                     alpha (the per-fragment state of the R&B
                                     buffer, Sec. 5.2) in the workspace, for a
                                     backward with RTGS_GRAD_SAVED_FRAGMENTS;
                                     needs RTGS_FWD_SAVE_STATE and a workspace
                                     sized with this flag (2 KB more per pair
                                     of capacity: room for every lane of a
                                     wave blending every list entry)          */
#define RTGS_FWD_BALANCE_LANES 32 /* assign each wave's 64 lanes the samples
                                     of similar work (the workload scheduling
                                     unit of Sec. 5.2): a tile's samples are
                                     sorted by the list entries each walked in
                                     a previous forward (session lane_work),
                                     waves take 64 consecutive ranks and cull
                                     against their samples' bounding box;
                                     writes this forward's walked entries to
                                     lane_work_out; render_fwd_batched only   */

/* ---- render_bwd flags ---- */
#define RTGS_GRAD_POSE        1   /* write g_pose6 and/or g_viewmat            */
#define RTGS_GRAD_MAP         2   /* write the five per-Gaussian gradients     */
#define RTGS_GRAD_COV3D       4   /* also write g_cov3d (needs RTGS_GRAD_MAP)  */
#define RTGS_GRAD_RECOMPUTE_STATE 8 /* final_T/last_idx were not saved: the
                                       backward recomputes them first          */
#define RTGS_GRAD_SAVED_FRAGMENTS 32 /* the forward saved its fragments
                                     (RTGS_FWD_SAVE_FRAGMENTS): the backward
                                     reads each blended fragment's alpha
                                     instead of re-evaluating Eq. 2, and skips
                                     list entries no pixel of a wave blended;
                                     the gradients are bitwise those without
                                     the flag                                 */
#define RTGS_GRAD_BALANCED_LANES 64 /* the forward used RTGS_FWD_BALANCE_LANES */
#define RTGS_GRAD_ADAM      128   /* with RTGS_GRAD_MAP, render_bwd_batched
                                     only: after each Gaussian's gradients,
                                     apply its session's Adam update
                                     (rtgs_session.adam) to its parameters in
                                     place, in the same pass (Sec. 3.1: the
                                     mapping update); the five gradient
                                     outputs may then be NULL                 */
#define RTGS_GRAD_SCORE      16   /* without RTGS_GRAD_MAP: write g_means and
                                     g_cov3d only, the inputs of the
                                     importance score of Sec. 4.1 (the raster
                                     pass of the pose-only backward); a
                                     session passing neither is skipped       */

/* ---- downsampled rendering (Sec. 4.2) ----
 * A frame downsampled to one pixel in 2^j (j = 2, 3, 4; 1 also accepted) is
 * rendered with one sample per block of 2^ceil(j/2) x 2^floor(j/2) pixels:
 * tiles of 16x16 samples, so the work scales with the samples, not the
 * pixels.  The sample of each block is the first pixel (raster order) the
 * pixel mask keeps in it; downsample_mask with the same j keeps exactly one.
 * All other pixels render as background (0, final_T = 1, last_idx = -1).
 * Per pixel the result equals rendering with that pixel mask at j = 0.
 * Single-session calls pass j in bits 8..11 of flags / grad_flags
 * (RTGS_SAMPLE_LOG2(j)); batched calls use rtgs_session.sample_log2.  The
 * forward and its backward must use the same j.  Workspace sizes computed
 * with j = 0 suffice for any j. */
#define RTGS_SAMPLE_SHIFT     8
#define RTGS_SAMPLE_LOG2(j)   ((j) << RTGS_SAMPLE_SHIFT)

/* ---- query states (Sec. 5.5: IDLE / EXECUTING) ---- */
#define RTGS_STATE_IDLE       0
#define RTGS_STATE_EXECUTING  1

#define RTGS_MAX_SESSIONS     64

typedef struct rtgs_context* rtgs_handle_t;

/* A Gaussian map (Eq. 1: mean, covariance via log-scales + quaternion,
 * opacity via its logit, colour).  gauss_mask may be NULL; a nonzero entry
 * excludes that Gaussian from rendering (the mask of the mask-prune step,
 * Sec. 4.1). */
typedef struct {
  const float* means;
  const float* log_scales;
  const float* quats;
  const float* opacity_logits;
  const float* colors;
  const uint8_t* gauss_mask;
  int32_t n;
} rtgs_gaussians;

/* Pinhole camera.  Intrinsics are host values; viewmat is a device pointer so
 * a pose optimised on the device needs no host round trip. */
typedef struct {
  int32_t width;
  int32_t height;
  float fx, fy, cx, cy;
  const float* viewmat;  /* device, 12 floats, row-major [R | t] */
} rtgs_camera;

/* Adam state of one session's map for RTGS_GRAD_ADAM (a HOST struct; the
 * arrays are device arrays of the parameters' shapes, updated in place).
 * Index order: means, log_scales, quats, opacity_logits, colors.  The update
 * is adam_step's, element for element and bitwise, on the float32 gradients
 * render_bwd would write: with t = step,
 *   m <- beta1 m + (1 - beta1) g,  v <- beta2 v + (1 - beta2) g^2,
 *   p <- p - (lr / (1 - beta1^t)) m / (sqrt(v) / sqrt(1 - beta2^t) + eps),
 * p being the session's map arrays (rtgs_gaussians), which the call writes.
 * Errors (INVALID_ARG): null moment array with n > 0, step < 1, a beta
 * outside [0, 1), eps < 0 or not finite, lr not finite. */
typedef struct {
  float* exp_avg[5];
  float* exp_avg_sq[5];
  float lr[5];
  int32_t step;                /* >= 1: the count of this update */
  double beta1, beta2, eps;
} rtgs_map_adam;

/* The loss gradient of a frame, formed by the forward that renders it (a
 * HOST struct of device arrays; see rtgs_session.l1).  The outputs are those
 * of loss_l1_grad(color, depth, target_color, target_depth, the session's
 * pixel_mask, n_active_dev, width, height, w_color, w_depth, dL_dcolor,
 * dL_ddepth) called on the forward's colour and depth, bitwise, for every
 * pixel of the frame.  Errors (INVALID_ARG): a null array, a pixel mask
 * without n_active_dev, weights not finite. */
typedef struct {
  const float* target_color;   /* [3][H][W] */
  const float* target_depth;   /* [H][W] */
  const int32_t* n_active_dev; /* device int32 (values below 1 count as 1), or
                                  NULL: W * H; required with a pixel mask */
  float w_color, w_depth;
  float* dL_dcolor;            /* [3][H][W], written */
  float* dL_ddepth;            /* [H][W], written */
} rtgs_l1_loss;

/* One session of a batched call: its own map, camera, masks, outputs and
 * gradients; same meaning as the arguments of render_fwd / render_bwd. */
typedef struct {
  rtgs_gaussians g;
  rtgs_camera cam;
  const uint8_t* pixel_mask;   /* [H][W] or NULL (all pixels active) */
  int32_t sample_log2;         /* 0, or j of a downsampled frame (see above) */
  /* forward outputs */
  float* color;                /* [3][H][W] */
  float* depth;                /* [H][W] expected depth sum w z */
  float* alpha;                /* [H][W] 1 - final_T */
  float* final_T;              /* [H][W] saved transmittance */
  int32_t* last_idx;           /* [H][W] position of the last blended pair, -1 */
  uint8_t* visible;            /* [n] 1 if projected and on screen, or NULL */
  int32_t* stats;              /* [3][H][W] with RTGS_FWD_STATS: fragments
                                  blended; list entries visited up to the stop
                                  (or the list end); list entries up to the
                                  last blended one.  NULL otherwise. */
  /* backward inputs */
  const float* dL_dcolor;      /* [3][H][W] */
  const float* dL_ddepth;      /* [H][W] */
  const float* dL_dalpha;      /* [H][W] or NULL */
  /* backward outputs (any may be NULL when its flag is off) */
  float* g_means;              /* [n][3] */
  float* g_log_scales;         /* [n][3] */
  float* g_quats;              /* [n][4] */
  float* g_opacity_logits;     /* [n] */
  float* g_colors;             /* [n][3] */
  float* g_pose6;              /* [6] (rho, phi) */
  float* g_viewmat;            /* [12] dL/d(viewmat entries), row-major 3x4 */
  float* g_cov3d;              /* [n][6] (xx, xy, xz, yy, yz, zz) */
  /* lane scheduling (RTGS_FWD_BALANCE_LANES; ignored without it) */
  const uint16_t* lane_work;   /* [H][W] lane_work_out of an earlier forward of
                                  this frame geometry, or NULL (then samples
                                  keep their index order, rows of 4 per wave) */
  uint16_t* lane_work_out;     /* [H][W] list entries each sample walked (at
                                  its block's first pixel), or NULL          */
  /* fused map update (RTGS_GRAD_ADAM; ignored without it) */
  const rtgs_map_adam* adam;   /* HOST pointer, or NULL: no update of this
                                  session's map                              */
  /* loss gradient formed by render_fwd_batched (Eq. 6; NULL: none) */
  const rtgs_l1_loss* l1;      /* HOST pointer, or NULL                      */
} rtgs_session;

/* Last error message of the calling thread (static storage, never NULL). */
const char* rtgs_last_error(void);

/* Create / destroy a handle bound to a HIP device. */
int32_t rtgs_create(rtgs_handle_t* out, int32_t device);
int32_t rtgs_destroy(rtgs_handle_t h);

/* Bytes of workspace for one session of n Gaussians at width x height with
 * room for pair_capacity (tile, Gaussian) pairs; flags are render_fwd flags.
 * `bytes` is a HOST pointer. */
int32_t rtgs_workspace_size(int32_t n, int32_t width, int32_t height,
                            int64_t pair_capacity, int32_t flags,
                            uint64_t* bytes);

/* Same for a batch; n, width, height are HOST arrays of n_sessions. */
int32_t rtgs_workspace_size_batched(const int32_t* n, const int32_t* width,
                                    const int32_t* height, int32_t n_sessions,
                                    int64_t pair_capacity, int32_t flags,
                                    uint64_t* bytes);

/* Forward pass (Steps 1-3, Sec. 2.1):
 *  1-1 projection: EWA linearisation of each Gaussian (Eq. 1) to a 2D mean,
 *      conic, opacity, colour and depth; Gaussians behind the near plane
 *      (z <= 0.2), masked, or with 255 * opacity < 1 are culled;
 *  1-2 tile intersection with 16x16 tiles;
 *  2   per-tile depth sort (ascending z, ties by Gaussian index);
 *  3   alpha (Eq. 2) and front-to-back blending (Eq. 3): alpha is clamped to
 *      0.99, fragments with alpha < 1/255 are skipped, a pixel stops before
 *      the fragment that would take T below 1e-4.
 * pixel_mask may be NULL; masked pixels render 0 with final_T = 1.
 * final_T and last_idx are written when RTGS_FWD_SAVE_STATE is set (they may
 * be NULL otherwise); visible may be NULL.
 * RTGS_FWD_REUSE_LISTS (the reuse of tile intersection and sorting across the
 * iterations of a frame, Sec. 3, Observation 6): Step 1-1 runs for the
 * current pose and parameters, Steps 1-2 and 2 are skipped and the tile
 * lists, depth order, tile rectangles and pair slots of the last forward
 * without this flag on the same workspace are used (a Gaussian that has
 * moved into a tile it was not listed for does not reach it; the lists keep
 * their reference depth order).  The caller guarantees that forward used the
 * same sessions, Gaussian counts, image sizes, sample_log2 and
 * pair_capacity; visible then reports the reference visibility.
 * Errors: INVALID_ARG (null required pointer, n < 0, W or H <= 0,
 * pair_capacity < 0, bad flags), WORKSPACE (ws_bytes too small), HIP. */
int32_t render_fwd(rtgs_handle_t h, const rtgs_gaussians* g,
                   const rtgs_camera* cam, const uint8_t* pixel_mask,
                   void* ws, uint64_t ws_bytes, int64_t pair_capacity,
                   float* out_color, float* out_depth, float* out_alpha,
                   float* final_T, int32_t* last_idx, uint8_t* visible_out,
                   int32_t flags, void* stream);

/* Backward pass (Steps 4-5, Sec. 2.2): the compositing in reverse from the
 * saved final_T and last_idx (or recomputed with RTGS_GRAD_RECOMPUTE_STATE),
 * per-pixel gradients merged per Gaussian, then pushed through the projection
 * to the map parameters and to the pose.  The pose gradient is the derivative
 * with respect to xi = (rho, phi) of Exp(xi) * viewmat at xi = 0 (left
 * perturbation; rho translation, phi rotation).  g_viewmat is the gradient
 * with respect to the 12 entries of viewmat taken as independent variables
 * (dL/dR = sum_k dL/dp_k mu_k^T + covariance term, dL/dt = sum_k dL/dp_k),
 * from which g_pose6 follows: rho part dL/dt, phi part the axial vector of
 * the antisymmetric part of dL/dR R^T + dL/dt t^T.  With RTGS_GRAD_POSE at
 * least one of g_pose6, g_viewmat must be non-NULL.  g_cov3d is dL/dSigma of the
 * world-frame covariance (symmetric, stored as xx, xy, xz, yy, yz, zz), the
 * input of the importance score.  dL_dalpha may be NULL.
 * The arguments g, cam, pixel_mask, ws and pair_capacity must be those of the
 * render_fwd whose results are being differentiated.
 * Errors: as render_fwd; RTGS_GRAD_ADAM is INVALID_ARG here (the fused
 * update takes render_bwd_batched, whose sessions carry the Adam state). */
int32_t render_bwd(rtgs_handle_t h, const rtgs_gaussians* g,
                   const rtgs_camera* cam, const uint8_t* pixel_mask,
                   void* ws, uint64_t ws_bytes, int64_t pair_capacity,
                   const float* final_T, const int32_t* last_idx,
                   const float* dL_dcolor, const float* dL_ddepth,
                   const float* dL_dalpha, int32_t grad_flags,
                   float* g_means, float* g_log_scales, float* g_quats,
                   float* g_opacity_logits, float* g_colors, float* g_pose6,
                   float* g_viewmat, float* g_cov3d, void* stream);

/* Batched forward / backward over n_sessions (<= RTGS_MAX_SESSIONS): one
 * launch per stage for all sessions, one tile space and one sort.  `sessions`
 * is a HOST array; each entry has the meaning of the single-session
 * arguments.  Per-session results equal those of single-session calls.  A
 * forward session with a non-NULL l1 also gets the gradient of the loss of
 * Eq. 6 with respect to its colour and depth (rtgs_l1_loss), written by the
 * rasterizer as it writes the image, so that no separate loss pass reads the
 * image back. */
int32_t render_fwd_batched(rtgs_handle_t h, const rtgs_session* sessions,
                           int32_t n_sessions, void* ws, uint64_t ws_bytes,
                           int64_t pair_capacity, int32_t flags, void* stream);
int32_t render_bwd_batched(rtgs_handle_t h, const rtgs_session* sessions,
                           int32_t n_sessions, void* ws, uint64_t ws_bytes,
                           int64_t pair_capacity, int32_t grad_flags,
                           void* stream);

/* Gradient of the tracking / mapping loss (Eq. 6, reading: L1 colour plus
 * w_depth times L1 depth, each a mean over the active pixels) with respect
 * to the rendered frame:
 *   dL/dC[c][p] = w_color * m_p * sign(C - C^) / (3 N)
 *   dL/dD[p]    = w_depth * m_p * sign(D - D^) / N,     sign(0) = 0,
 * m_p = pixel_mask[p] != 0 (1 when pixel_mask is NULL); N = *n_active_dev
 * (a device int32, e.g. the count downsample_mask writes; values below 1
 * count as 1), or W * H when n_active_dev is NULL.  All arrays are device
 * arrays: colours [3][H][W], depths and mask [H][W]; outputs overwritten.
 * Errors: INVALID_ARG (null array, W or H <= 0, a mask without n_active_dev,
 * weights not finite), HIP. */
int32_t loss_l1_grad(const float* color, const float* depth,
                     const float* target_color, const float* target_depth,
                     const uint8_t* pixel_mask, const int32_t* n_active_dev,
                     int32_t width, int32_t height, float w_color,
                     float w_depth, float* dL_dcolor, float* dL_ddepth,
                     void* stream);

/* loss_l1_grad for several frames (e.g. the sessions of one batched
 * iteration): items is a HOST array of n_items; each entry has the meaning
 * of the single-frame arguments (its own size, mask and count).  One launch
 * per 32 items.  Errors: as loss_l1_grad. */
typedef struct rtgs_loss_item {
  const float* color;
  const float* depth;
  const float* target_color;
  const float* target_depth;
  const uint8_t* pixel_mask;
  const int32_t* n_active_dev;
  float* dL_dcolor;
  float* dL_ddepth;
  int32_t width;
  int32_t height;
} rtgs_loss_item;

int32_t loss_l1_grad_batched(const rtgs_loss_item* items, int32_t n_items,
                             float w_color, float w_depth, void* stream);

/* Parameter update of the mapping stage: the Gaussian gradients of Step 5
 * update the 3D Gaussian parameters (Sec. 3.1).  The paper names no
 * optimiser; this is Adam without weight decay.  For each group (a HOST
 * array of n_groups entries; every pointer in an entry is a device float
 * array of n elements, updated in place):
 *   exp_avg    <- beta1 exp_avg + (1 - beta1) grad
 *   exp_avg_sq <- beta2 exp_avg_sq + (1 - beta2) grad^2
 *   param      <- param - lr / (1 - beta1^step) * exp_avg
 *                        / (sqrt(exp_avg_sq) / sqrt(1 - beta2^step) + eps)
 * where step (>= 1) is the group's update count including this one; the
 * arithmetic is float32, with 1 - beta and the two bias factors formed in
 * double on the host.  Groups
 * may be tensors of different sessions; all of them are updated by one
 * kernel launch per 64 groups.  Groups must not overlap.  Errors:
 * INVALID_ARG (null array with n > 0, n < 0, step < 1, beta outside [0, 1),
 * eps < 0 or not finite, lr not finite), HIP. */
typedef struct rtgs_adam_group {
  float* param;
  const float* grad;
  float* exp_avg;
  float* exp_avg_sq;
  int64_t n;
  float lr;
  int32_t step;
} rtgs_adam_group;

int32_t adam_step(rtgs_handle_t h, const rtgs_adam_group* groups,
                  int32_t n_groups, double beta1, double beta2, double eps,
                  void* stream);

/* Pose update of the tracking stage (Sec. 3.1: tracking updates the camera
 * pose; Step 5 gives dL/dP).  For each item (a HOST array of n; every
 * pointer is a device float array): Adam on the left-perturbation tangent
 * xi = (rho, phi) at xi = 0 with the gradient g_pose6 (as render_bwd writes
 * it),
 *   m <- beta1 m + (1 - beta1) g,   v <- beta2 v + (1 - beta2) g^2,
 *   s_i = lr_i (m_i / (1 - beta1^step)) / (sqrt(v_i / (1 - beta2^step)) + eps)
 * (lr_i = lr_rho for rho, lr_phi for phi), then the re-linearisation
 *   viewmat <- Exp(-s) viewmat
 * (xi returns to zero).  Arithmetic in float64; viewmat [12] row-major 3x4,
 * exp_avg / exp_avg_sq [6] updated in place.  step (>= 1) counts this
 * update.  One launch per 48 items.  Errors: INVALID_ARG, HIP. */
typedef struct rtgs_pose_item {
  float* viewmat;
  const float* g_pose6;
  float* exp_avg;
  float* exp_avg_sq;
  float lr_rho;
  float lr_phi;
  int32_t step;
} rtgs_pose_item;

int32_t pose_update(const rtgs_pose_item* items, int32_t n, double beta1,
                    double beta2, double eps, void* stream);

/* Adaptive Gaussian pruning, the mask step (Sec. 4.1, Eq. 7):
 * score_k = ||dL/dmu_k||_2 + lambda * ||dL/dSigma_k||_F (Frobenius over the
 * nine entries of the symmetric gradient); among the V Gaussians with
 * visible != 0 and mask_in == 0, the floor(max_ratio * V) with the lowest
 * (score, index) are added to the mask: mask_out = mask_in | selected.
 * visible and mask_in may be NULL (all visible / none masked).
 * n_masked_dev (device int32) receives the number newly masked; score_out
 * (device float [n]) may be NULL.  Requires 0 <= max_ratio <= 0.5 (the
 * paper's 50% cap, Sec. 6.2); lambda defaults to 0.8 in the paper.
 * Errors: INVALID_ARG, HIP. */
int32_t prune_by_grad(rtgs_handle_t h, const float* g_means,
                      const float* g_cov3d, const uint8_t* visible,
                      const uint8_t* mask_in, int32_t n, float lambda,
                      float max_ratio, uint8_t* mask_out,
                      int32_t* n_masked_dev, float* score_out, void* stream);

/* Mask-prune schedule (Sec. 4.1): Gaussians masked for K iterations are then
 * permanently removed.  compact_by_mask copies the rows i with drop[i] == 0
 * of each item, in index order, to the front of its dst: row k of dst is
 * the k-th kept row of src.  items is a HOST array of n_items
 * (<= RTGS_COMPACT_MAX_ITEMS); src is a device array of n rows of row_bytes
 * (> 0) each, dst one of dst_rows rows (kept rows past dst_rows are not
 * written), the two not overlapping, 4-byte aligned when row_bytes is a
 * multiple of 4.
 * drop: device uint8 [n]; n_kept (device int32) receives the kept count.
 * scratch: device memory of rtgs_compact_scratch_size(n) bytes.  n = 0 is a
 * no-op that writes n_kept = 0 (src and dst may then be NULL).
 * Errors: INVALID_ARG, WORKSPACE, HIP. */
#define RTGS_COMPACT_MAX_ITEMS 24
typedef struct rtgs_compact_item {
  const void* src;
  void* dst;
  int32_t row_bytes;
  int32_t dst_rows;
} rtgs_compact_item;

uint64_t rtgs_compact_scratch_size(int32_t n);
int32_t compact_by_mask(const uint8_t* drop, int32_t n,
                        const rtgs_compact_item* items, int32_t n_items,
                        void* scratch, uint64_t scratch_bytes,
                        int32_t* n_kept, void* stream);

/* compact_by_mask without allocation and without a caller scratch, for
 * callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation).  Same arguments,
 * result and errors as compact_by_mask, without scratch / scratch_bytes; the
 * library's own device scratch (64 KB per GPU, a static device array held
 * until the process ends) limits n to RTGS_COMPACT_STATIC_MAX_ROWS: larger n
 * returns RTGS_ERR_WORKSPACE.  No memory is allocated or freed; the first
 * call on a GPU looks up the scratch's address there.  The stream must belong
 * to the current device (else RTGS_ERR_INVALID_ARG).  Every call on one GPU
 * shares that scratch: calls that overlap on one GPU (other streams, other
 * threads) race and must be serialised by the caller. */
#define RTGS_COMPACT_STATIC_MAX_ROWS 16776192   /* (16384 - 1) * 1024 */
int32_t compact_by_mask_static(const uint8_t* drop, int32_t n,
                               const rtgs_compact_item* items, int32_t n_items,
                               int32_t* n_kept, void* stream);

/* The tile rectangle of every Gaussian after a full render_fwd on ws (the
 * same n, width, height, sample_log2 and pair_capacity as that call):
 * rect_out (device int32 [n][4]) = (x0, y0, x1, y1) in tiles, inclusive,
 * x1 < x0 for a Gaussian that touches no tile.  The Gaussian's pairs are
 * exactly the tiles of its rectangle.  Errors: INVALID_ARG, WORKSPACE, HIP. */
int32_t rtgs_tile_rects(int32_t n, int32_t width, int32_t height,
                        int32_t sample_log2, int64_t pair_capacity,
                        const void* ws, uint64_t ws_bytes, int32_t* rect_out,
                        void* stream);

/* Change of the tile-Gaussian intersections between two sets of rectangles
 * (Sec. 4.1: the ratio that sets the next pruning interval): out (device
 * int64 [2]) receives out[0] = sum over Gaussians i with skip[i] == 0 of the
 * tiles in exactly one of rect_ref[i] and rect_cur[i], out[1] = sum of the
 * tiles of rect_ref[i]; the ratio is out[0] / out[1].  skip may be NULL.
 * Errors: INVALID_ARG, HIP. */
int32_t tile_pair_change(const int32_t* rect_ref, const int32_t* rect_cur,
                         const uint8_t* skip, int32_t n, int64_t* out,
                         void* stream);

/* Dynamic downsampling (Sec. 4.2) as a pixel mask: keep 1 pixel in 2^j,
 * one per block of 2^ceil(j/2) x 2^floor(j/2) pixels (4x4, 4x2, 2x2 for
 * j = 4, 3, 2; ragged blocks at the right and bottom edges), choosing the
 * pixel with the lowest final_T of the previous forward (ties to the lowest
 * raster index).  j = 0 keeps every pixel.  n_active_dev (device int32, may
 * be NULL) receives the number of kept pixels.  0 <= log2_ratio <= 8.
 * Errors: INVALID_ARG, HIP. */
int32_t downsample_mask(const float* final_T, int32_t width, int32_t height,
                        int32_t log2_ratio, uint8_t* mask_out,
                        int32_t* n_active_dev, void* stream);

/* The downsampling schedule of Sec. 4.2 (host only): 0 for a keyframe; for
 * non-keyframe n after keyframe k, the pixel ratio min(2^-4 m^(n-k-1), 2^-2)
 * as j = max(2, 4 - floor((n - k - 1) log2 m)).  Returns j, or
 * RTGS_ERR_INVALID_ARG if n <= k for a non-keyframe or m < 2. */
int32_t rtgs_downsample_log2_ratio(int32_t is_keyframe, int32_t n, int32_t k,
                                   int32_t m);

/* Status (Sec. 5.5, the check-status call): with blocking != 0 waits for the
 * work enqueued through h, then reports in *pairs_needed (HOST, may be NULL)
 * the largest pair count any render_fwd needed since the previous query, and
 * resets.  Returns RTGS_ERR_CAPACITY if any of those calls needed more pairs
 * than the capacity it was given (then *pairs_needed is the largest such
 * need).  With blocking == 0 and work pending, *state = RTGS_STATE_EXECUTING
 * and nothing is reset. */
int32_t rtgs_query(rtgs_handle_t h, int32_t blocking, int64_t* pairs_needed,
                   int32_t* state);

/* Test access to forward intermediates kept in a workspace after render_fwd.
 * n, width, height, sample_log2 (HOST arrays of n_sessions; sample_log2 may
 * be NULL for all zero) and pair_capacity must be those of that call.  All outputs are device arrays and any may be NULL: per
 * Gaussian of the batch (global index over sessions)
 *   stage [n][12] = u, v, conic a, b, c, opacity, depth z, e_x, e_y,
 *                   r, g, b   (u, v: float32 part of the centre; e_x, e_y:
 *                   half-widths of the bounding box of the alpha = 1/255
 *                   ellipse, Step 1-2)
 *   rect [n][4]   = tile rectangle x0, y0, x1, y1 (x1 < x0 when empty)
 * per tile of the batch: ranges [T][2] = [start, end) into ids; ids [P] =
 * Gaussian ids in tile-then-depth order (at most ids_capacity written). */
int32_t rtgs_debug_stage(const int32_t* n, const int32_t* width,
                         const int32_t* height, const int32_t* sample_log2,
                         int32_t n_sessions,
                         int64_t pair_capacity, const void* ws,
                         uint64_t ws_bytes, float* stage, int32_t* rect,
                         int32_t* ranges, int32_t* ids, int64_t ids_capacity,
                         void* stream);

/* Stage profiler (HIP events on the stream each kernel is launched on).
 * Stages: 0 init, 1 preprocess, 2 scan, 3 emit, 4 sort, 5 raster_fwd,
 * 6 adam, 7 raster_bwd, 8 preprocess_bwd (with RTGS_GRAD_ADAM also the
 * map's Adam update), 9 pose_reduce, 10 bin_count, 11 merge.  After
 * rtgs_profile_enable(h, mask) every launch of a stage whose bit is set is
 * bracketed by two events; rtgs_profile_read waits for them and returns per
 * stage the summed milliseconds and the launch count (HOST arrays of
 * RTGS_PROFILE_STAGES entries), then clears.  mask = 0 disables. */
#define RTGS_PROFILE_STAGES 16
int32_t rtgs_profile_enable(rtgs_handle_t h, int32_t stage_mask);
int32_t rtgs_profile_read(rtgs_handle_t h, double* total_ms, int64_t* launches);

/* Test hook for the wavefront reduce-scatter of the backward merge (ten
 * values per lane, as in the full-gradient backward): for each wave w of
 * n_waves and value i < 10, out[10 w + i] = sum over lanes l < 64 of
 * in[(10 w + i) * 64 + l].  in and out are device arrays. */
int32_t rtgs_selftest_wave_sum(const float* in, float* out, int32_t n_waves,
                               void* stream);

#ifdef __cplusplus
}
#endif
#endif /* RTGS_H */
