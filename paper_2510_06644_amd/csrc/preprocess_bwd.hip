// Step 5, preprocessing backpropagation (Sec. 2.2): the per-Gaussian 2D
// gradients merged by the raster backward are pushed through the EWA
// projection to the map parameters, and in tracking summed over Gaussians to
// the camera-pose gradient dL/dP (the paper's Preprocessing Engine and
// Merging Tree, Secs. 5.1 and 5.4).  In mapping the Adam update of the map
// (Sec. 3.1) can follow in the same pass.
//
// Two kernels.  The tile -> Gaussian merge (the role of the paper's Stage
// Buffer): each Gaussian's 2D gradient is the fixed-order sum of its
// (tile, Gaussian) pair slots, 40 B each; a streaming kernel at full
// occupancy.  Then one thread per Gaussian in float64 through the
// projection (56 B of parameters and 40 B of merged gradient in), writing
// the gradients (56 B) or, fused, applying Adam to the Gaussian's 14
// parameters right away (parameters and both moments read and written,
// 280 B), so the gradients never go through memory.  That kernel needs many
// float64 registers, hence few waves: the merge stays apart, where
// occupancy hides its loads.  The pose partials are summed per workgroup in
// LDS, then per session in a fixed order by a third kernel, so the pose
// reduction adds no float atomics of its own.
//
// Chain (all derivatives exact for the forward of forward_prep.hip):
//   conic (a, b, c) -> Sigma' :  dL/dSigma' = -M G_M M,  G_M = [[ga, gb/2],
//                                [gb/2, gc]]
//   Sigma' = A A^T + 0.3 I, A = T M, T = J W, M = R diag(s):
//     dL/dA = 2 G' A,  dL/dM = T^T dL/dA,  dL/dT = dL/dA M^T
//   T = J W:  dL/dJ = dL/dT W^T,  dL/dW|cov = J^T dL/dT
//   J(p), u(p), v(p), z: dL/dp;  dL/dmu = W^T dL/dp
//   view matrix [W | t]: dL/dW = dL/dW|cov + dL/dp mu^T, dL/dt = dL/dp,
//     summed over Gaussians; the pose (left perturbation at xi = 0) is then
//     dL/drho = dL/dt and dL/dphi = the axial vector of the antisymmetric
//     part of A = dL/dW W^T + dL/dt t^T: (A21 - A12, A02 - A20, A10 - A01)
//   M -> scales (dL/dl = s dL/ds) and R(q/|q|) -> quaternion.
#include "rtgs_internal.h"

namespace rtgs {
namespace {

// Tile -> Gaussian merge: kMergeLanes lanes (part of a DPP row) per Gaussian
// sum its pair slots, strided, then a fixed DPP tree; the last of them stores
// the NV totals.  A Gaussian with more than kMergeBig slots (a few hundred of 300k
// touch up to ~1400 tiles) would make its row the kernel's critical path, so
// its row hands it to the whole workgroup, whose 256 lanes sum it after the
// rows are done.  Every sum is in a fixed order: deterministic.
constexpr int kMergeBig = 128;
constexpr int kMergeLanes = 8;            // lanes per Gaussian (a half DPP row)
constexpr int kMergePerBlock = 256 / kMergeLanes;

// Lane `lane` of `width` adds slots lane, lane + width, ... of the n slots at
// `first`; four slots are loaded per round, so that a long list does not
// serialise on one load at a time.
template <int NV>
__device__ __forceinline__ void sum_slots(const WsPtrs& W, int64_t first, int64_t n, int lane,
                                          int width, float (&acc)[NV]) {
  for (int64_t k0 = lane; k0 < n; k0 += 4 * width) {
    float v[4][NV];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t k = k0 + (int64_t)width * j;
      // a slot is NV floats at an 8-byte aligned offset: NV / 2 8-byte loads
      const float2* p = reinterpret_cast<const float2*>(W.partial + (first + k) * NV);
#pragma unroll
      for (int i = 0; i < NV / 2; ++i) {
        const float2 x = k < n ? p[i] : make_float2(0.f, 0.f);
        v[j][2 * i] = x.x;
        v[j][2 * i + 1] = x.y;
      }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int i = 0; i < NV; ++i) acc[i] += v[j][i];
  }
}

// Sums over runs of LANES (8 or 16) lanes of each DPP row; the run's last
// lane holds its total.
template <int LANES, int NV>
__device__ __forceinline__ void row_sums(float (&acc)[NV]) {
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    float v = acc[i];
    v += dpp_f<kDppRowShr1, 0xf, true>(v);
    v += dpp_f<kDppRowShr2, 0xf, true>(v);
    v += dpp_f<kDppRowShr4, 0xf, true>(v);
    if (LANES == 16) v += dpp_f<kDppRowShr8, 0xf, true>(v);
    acc[i] = v;
  }
}

template <int NV>
__global__ __launch_bounds__(256) void k_merge(Batch B, WsPtrs W) {
  __shared__ int s_big[kMergePerBlock];
  __shared__ int s_nbig;
  __shared__ float s_row[16][NV];
  const int row = threadIdx.x >> 4;
  const int gid = blockIdx.x * kMergePerBlock + (int)threadIdx.x / kMergeLanes;
  const int sub = threadIdx.x % kMergeLanes;
  if (threadIdx.x == 0) s_nbig = 0;
  __syncthreads();
  float acc[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) acc[i] = 0.f;
  bool mine = gid < B.n_total;
  if (mine) {
    const int64_t first = W.goff[gid];
    // slots past the pair capacity were never written
    const int64_t n = min((int64_t)W.cnt[gid], W.cap - first);
    if (n > kMergeBig) {
      mine = false;
      if (sub == 0) s_big[atomicAdd(&s_nbig, 1)] = gid;
    } else {
      sum_slots<NV>(W, first, n, sub, kMergeLanes, acc);
    }
  }
  row_sums<kMergeLanes, NV>(acc);
  if (sub == kMergeLanes - 1 && mine) {
    float* d = W.grad2d + (int64_t)gid * 10;
#pragma unroll
    for (int i = 0; i < NV; ++i) d[i] = acc[i];
  }
  __syncthreads();
  const int nbig = s_nbig;
  for (int q = 0; q < nbig; ++q) {
    // s_big's order depends on timing; each Gaussian's sum does not
    const int g = s_big[q];
    const int64_t first = W.goff[g];
    const int64_t n = min((int64_t)W.cnt[g], W.cap - first);
#pragma unroll
    for (int i = 0; i < NV; ++i) acc[i] = 0.f;
    sum_slots<NV>(W, first, n, (int)threadIdx.x, 256, acc);
    row_sums<16, NV>(acc);
    if ((threadIdx.x & 15) == 15)
#pragma unroll
      for (int i = 0; i < NV; ++i) s_row[row][i] = acc[i];
    __syncthreads();
    if (threadIdx.x < NV) {
      float t = 0.f;
      for (int r = 0; r < 16; ++r) t += s_row[r][threadIdx.x];
      W.grad2d[(int64_t)g * 10 + threadIdx.x] = t;
    }
    __syncthreads();                      // s_row is reused by the next one
  }
}

template <int NV, bool ADAM, bool ONE>
__global__ __launch_bounds__(kGaussPerBlock) void k_gauss_bwd(Batch B, WsPtrs W, int flags) {
  __shared__ double s_red[kGaussPerBlock / 64][12];
  const int s = ONE ? 0 : find_session(session_table(B), B.n_sessions, (int)blockIdx.x,
                                       [](const SessionDev& x) { return x.block_base; });
  const SessionDev& S = batch_session<ONE>(B, s);
  const int li0 = ((int)blockIdx.x - S.block_base) * kGaussPerBlock;
  // ---- projection backward, one thread per Gaussian
  const int li = li0 + (int)threadIdx.x;
  const bool want_map = (flags & RTGS_GRAD_MAP) != 0;
  const bool want_cov = (flags & RTGS_GRAD_COV3D) != 0 && S.g_cov3d != nullptr;
  // score inputs only (dL/dmu, dL/dSigma) on the pose-only raster path
  const bool want_score = !want_map && (flags & RTGS_GRAD_SCORE) != 0 && S.g_means != nullptr &&
                          S.g_cov3d != nullptr;
  double pose[12] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};   // dL/dW (9), dL/dt (3)
  if (li < S.n) {
    const int gid = S.gauss_base + li;
    const int4 rect = W.rect[gid];
    double gm[3] = {0, 0, 0}, gl[3] = {0, 0, 0}, gq[4] = {0, 0, 0, 0}, go_eta = 0;
    double gcol[3] = {0, 0, 0}, gsig[6] = {0, 0, 0, 0, 0, 0};
    if (rect.z >= rect.x) {
      // the merged 2D gradient: (u, v, a, b, c, o, r, g, b, z), or with the
      // pose-only merge (u, v, a, b, c, z)
      float g2[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
      const float* m = W.grad2d + (int64_t)gid * 10;
      if (NV == 10) {
        for (int i = 0; i < 10; ++i) g2[i] = m[i];
      } else {
        for (int i = 0; i < 5; ++i) g2[i] = m[i];
        g2[9] = m[5];
      }
      const double gu = g2[0], gv = g2[1], ga = g2[2], gb = g2[3], gc = g2[4], go = g2[5];
      gcol[0] = g2[6]; gcol[1] = g2[7]; gcol[2] = g2[8];
      const double gdep = g2[9];
      double vm[12];
      for (int k = 0; k < 12; ++k) vm[k] = S.viewmat[k];
      const double mx = S.means[3 * li], my = S.means[3 * li + 1], mz = S.means[3 * li + 2];
      const double qw = S.quats[4 * li], qx = S.quats[4 * li + 1];
      const double qy = S.quats[4 * li + 2], qz = S.quats[4 * li + 3];
      double sc[3], o;
      activate(S, li, sc, o);
      const double x = vm[0] * mx + vm[1] * my + vm[2] * mz + vm[3];
      const double y = vm[4] * mx + vm[5] * my + vm[6] * mz + vm[7];
      const double z = vm[8] * mx + vm[9] * my + vm[10] * mz + vm[11];
      // reciprocals taken once (a float64 division is a long instruction sequence)
      const double qn = sqrt(qw * qw + qx * qx + qy * qy + qz * qz), iqn = 1.0 / qn;
      const double w = qw * iqn, a = qx * iqn, b = qy * iqn, c = qz * iqn;
      const double R[9] = {1 - 2 * (b * b + c * c), 2 * (a * b - w * c), 2 * (a * c + w * b),
                           2 * (a * b + w * c), 1 - 2 * (a * a + c * c), 2 * (b * c - w * a),
                           2 * (a * c - w * b), 2 * (b * c + w * a), 1 - 2 * (a * a + b * b)};
      double M[9];
      for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) M[3 * r + k] = R[3 * r + k] * sc[k];
      const double limx = kFovClamp * 0.5 * S.width / S.fx;
      const double limy = kFovClamp * 0.5 * S.height / S.fy;
      const double iz = 1.0 / z, iz2 = iz * iz, iz3 = iz2 * iz;
      const double rx = x * iz, ry = y * iz;
      const bool inx = rx > -limx && rx < limx, iny = ry > -limy && ry < limy;
      const double tx = fmin(limx, fmax(-limx, rx)), ty = fmin(limy, fmax(-limy, ry));
      const double j00 = S.fx * iz, j02 = -S.fx * tx * iz, j11 = S.fy * iz, j12 = -S.fy * ty * iz;
      double T0[3], T1[3], A0[3], A1[3];
      for (int k = 0; k < 3; ++k) {
        T0[k] = j00 * vm[k] + j02 * vm[8 + k];
        T1[k] = j11 * vm[4 + k] + j12 * vm[8 + k];
      }
      for (int k = 0; k < 3; ++k) {
        A0[k] = T0[0] * M[k] + T0[1] * M[3 + k] + T0[2] * M[6 + k];
        A1[k] = T1[0] * M[k] + T1[1] * M[3 + k] + T1[2] * M[6 + k];
      }
      const double sxx = A0[0] * A0[0] + A0[1] * A0[1] + A0[2] * A0[2] + kDilation;
      const double sxy = A0[0] * A1[0] + A0[1] * A1[1] + A0[2] * A1[2];
      const double syy = A1[0] * A1[0] + A1[1] * A1[1] + A1[2] * A1[2] + kDilation;
      const double inv = 1.0 / (sxx * syy - sxy * sxy);
      const double ca = syy * inv, cb = -sxy * inv, cc = sxx * inv;
      // dL/dSigma' (symmetric matrix entries)
      const double Gxx = -(ga * ca * ca + gb * ca * cb + gc * cb * cb);
      const double Gyy = -(ga * cb * cb + gb * cb * cc + gc * cc * cc);
      const double Gxy = -(ga * ca * cb + 0.5 * gb * (ca * cc + cb * cb) + gc * cb * cc);
      double dA0[3], dA1[3], dM[9], dT0[3], dT1[3];
      for (int k = 0; k < 3; ++k) {
        dA0[k] = 2.0 * (Gxx * A0[k] + Gxy * A1[k]);
        dA1[k] = 2.0 * (Gxy * A0[k] + Gyy * A1[k]);
      }
      for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) dM[3 * r + k] = T0[r] * dA0[k] + T1[r] * dA1[k];
      for (int r = 0; r < 3; ++r) {
        dT0[r] = dA0[0] * M[3 * r] + dA0[1] * M[3 * r + 1] + dA0[2] * M[3 * r + 2];
        dT1[r] = dA1[0] * M[3 * r] + dA1[1] * M[3 * r + 1] + dA1[2] * M[3 * r + 2];
      }
      // T0 = j00 W0 + j02 W2, T1 = j11 W1 + j12 W2 (W rows)
      const double dj00 = dT0[0] * vm[0] + dT0[1] * vm[1] + dT0[2] * vm[2];
      const double dj02 = dT0[0] * vm[8] + dT0[1] * vm[9] + dT0[2] * vm[10];
      const double dj11 = dT1[0] * vm[4] + dT1[1] * vm[5] + dT1[2] * vm[6];
      const double dj12 = dT1[0] * vm[8] + dT1[1] * vm[9] + dT1[2] * vm[10];
      double dW[9];
      for (int k = 0; k < 3; ++k) {
        dW[k] = j00 * dT0[k];
        dW[3 + k] = j11 * dT1[k];
        dW[6 + k] = j02 * dT0[k] + j12 * dT1[k];
      }
      // dL/dp from u, v, J and the depth output
      double gx = gu * S.fx * iz + (inx ? dj02 * (-S.fx * iz2) : 0.0);
      double gy = gv * S.fy * iz + (iny ? dj12 * (-S.fy * iz2) : 0.0);
      const double dj02dz = S.fx * tx * iz2 + (inx ? S.fx * x * iz3 : 0.0);
      const double dj12dz = S.fy * ty * iz2 + (iny ? S.fy * y * iz3 : 0.0);
      double gz = gdep - gu * S.fx * x * iz2 - gv * S.fy * y * iz2 - dj00 * S.fx * iz2 -
                  dj11 * S.fy * iz2 + dj02 * dj02dz + dj12 * dj12dz;
      // view matrix: dL/dW = dL/dW|cov + dL/dp mu^T, dL/dt = dL/dp
      const double gp3[3] = {gx, gy, gz}, mu[3] = {mx, my, mz};
      for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) pose[3 * i + j] = dW[3 * i + j] + gp3[i] * mu[j];
        pose[9 + i] = gp3[i];
      }
      if (want_score) {
        for (int k = 0; k < 3; ++k) gm[k] = vm[k] * gx + vm[4 + k] * gy + vm[8 + k] * gz;
        double GT0[3], GT1[3];
        for (int k = 0; k < 3; ++k) {
          GT0[k] = Gxx * T0[k] + Gxy * T1[k];
          GT1[k] = Gxy * T0[k] + Gyy * T1[k];
        }
        const int ii[6] = {0, 0, 0, 1, 1, 2}, jj[6] = {0, 1, 2, 1, 2, 2};
        for (int k = 0; k < 6; ++k) gsig[k] = T0[ii[k]] * GT0[jj[k]] + T1[ii[k]] * GT1[jj[k]];
      }
      if (want_map) {
        // dL/dmu = W^T dL/dp
        for (int k = 0; k < 3; ++k) gm[k] = vm[k] * gx + vm[4 + k] * gy + vm[8 + k] * gz;
        // M = R diag(s): dR[r][k] = dM[r][k] s_k, ds_k = sum_r R[r][k] dM[r][k]
        double dR[9];
        for (int r = 0; r < 3; ++r)
          for (int k = 0; k < 3; ++k) dR[3 * r + k] = dM[3 * r + k] * sc[k];
        for (int k = 0; k < 3; ++k)
          gl[k] = sc[k] * (R[k] * dM[k] + R[3 + k] * dM[3 + k] + R[6 + k] * dM[6 + k]);
        // R(w, a, b, c) -> unit-quaternion gradient
        const double gw =
            2 * (-c * dR[1] + b * dR[2] + c * dR[3] - a * dR[5] - b * dR[6] + a * dR[7]);
        const double gx4 = 2 * (b * dR[1] + c * dR[2] + b * dR[3] - 2 * a * dR[4] - w * dR[5] +
                                c * dR[6] + w * dR[7] - 2 * a * dR[8]);
        const double gy4 = 2 * (-2 * b * dR[0] + a * dR[1] + w * dR[2] + a * dR[3] + c * dR[5] -
                                w * dR[6] + c * dR[7] - 2 * b * dR[8]);
        const double gz4 = 2 * (-2 * c * dR[0] - w * dR[1] + a * dR[2] + w * dR[3] - 2 * c * dR[4] +
                                b * dR[5] + a * dR[6] + b * dR[7]);
        const double dot = w * gw + a * gx4 + b * gy4 + c * gz4;
        gq[0] = (gw - w * dot) * iqn;
        gq[1] = (gx4 - a * dot) * iqn;
        gq[2] = (gy4 - b * dot) * iqn;
        gq[3] = (gz4 - c * dot) * iqn;
        go_eta = go * o * (1.0 - o);
        if (want_cov) {
          // dL/dSigma = T^T G' T
          double GT0[3], GT1[3];
          for (int k = 0; k < 3; ++k) {
            GT0[k] = Gxx * T0[k] + Gxy * T1[k];
            GT1[k] = Gxy * T0[k] + Gyy * T1[k];
          }
          const int ii[6] = {0, 0, 0, 1, 1, 2}, jj[6] = {0, 1, 2, 1, 2, 2};
          for (int k = 0; k < 6; ++k) gsig[k] = T0[ii[k]] * GT0[jj[k]] + T1[ii[k]] * GT1[jj[k]];
        }
      }
    }
    if (want_map) {
      if (S.g_means) for (int k = 0; k < 3; ++k) S.g_means[3 * li + k] = (float)gm[k];
      if (S.g_log_scales) for (int k = 0; k < 3; ++k) S.g_log_scales[3 * li + k] = (float)gl[k];
      if (S.g_quats) for (int k = 0; k < 4; ++k) S.g_quats[4 * li + k] = (float)gq[k];
      if (S.g_opac) S.g_opac[li] = (float)go_eta;
      if (S.g_colors) for (int k = 0; k < 3; ++k) S.g_colors[3 * li + k] = (float)gcol[k];
      if (want_cov) for (int k = 0; k < 6; ++k) S.g_cov3d[6 * li + k] = (float)gsig[k];
    }
    if (want_score) {
      for (int k = 0; k < 3; ++k) S.g_means[3 * li + k] = (float)gm[k];
      for (int k = 0; k < 6; ++k) S.g_cov3d[6 * li + k] = (float)gsig[k];
    }
    // ---- Adam on the Gaussian's parameters (the update of adam_step, on
    // the same float32 gradients).  The constants, then every parameter and
    // moment, are read before the first store: the stores may alias them, so
    // read element by element each would wait for the previous one's store.
    if (ADAM && S.adam.on) {
      const MapAdamDev& A = S.adam;
      const float beta1 = A.beta1, beta2 = A.beta2, omb1 = A.omb1, omb2 = A.omb2, eps = A.eps;
      const float isb2 = A.inv_sqrt_bc2;
      float step[5];
      float* par[5] = {const_cast<float*>(S.means), const_cast<float*>(S.log_scales),
                       const_cast<float*>(S.quats), const_cast<float*>(S.opac),
                       const_cast<float*>(S.colors)};
      float *pm[5], *pv2[5];
#pragma unroll
      for (int t = 0; t < 5; ++t) {
        step[t] = A.step_size[t];
        pm[t] = A.m[t];
        pv2[t] = A.v[t];
      }
      const float g14[14] = {(float)gm[0], (float)gm[1], (float)gm[2], (float)gl[0],
                             (float)gl[1], (float)gl[2], (float)gq[0], (float)gq[1],
                             (float)gq[2], (float)gq[3], (float)go_eta, (float)gcol[0],
                             (float)gcol[1], (float)gcol[2]};
      constexpr int kDim[5] = {3, 3, 4, 1, 3};
      float P[14], Mo[14], Vo[14];
      {
        int at = 0;
#pragma unroll
        for (int t = 0; t < 5; ++t) {
#pragma unroll
          for (int k = 0; k < kDim[t]; ++k) {
            const int64_t e = (int64_t)kDim[t] * li + k;
            P[at + k] = par[t][e];
            Mo[at + k] = pm[t][e];
            Vo[at + k] = pv2[t][e];
          }
          at += kDim[t];
        }
      }
      {
        int at = 0;
#pragma unroll
        for (int t = 0; t < 5; ++t) {
#pragma unroll
          for (int k = 0; k < kDim[t]; ++k)
            adam_update(P[at + k], g14[at + k], Mo[at + k], Vo[at + k], beta1, beta2, omb1, omb2,
                        eps, step[t], isb2);
          at += kDim[t];
        }
      }
      {
        int at = 0;
#pragma unroll
        for (int t = 0; t < 5; ++t) {
#pragma unroll
          for (int k = 0; k < kDim[t]; ++k) {
            const int64_t e = (int64_t)kDim[t] * li + k;
            par[t][e] = P[at + k];
            pm[t][e] = Mo[at + k];
            pv2[t][e] = Vo[at + k];
          }
          at += kDim[t];
        }
      }
    }
  }
  // block partial of the pose gradient: wave shuffles, then the 4 waves in LDS
  // (the flag is the launch's, so the whole workgroup leaves together)
  if (!(flags & RTGS_GRAD_POSE)) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int k = 0; k < 12; ++k) {
    double v = pose[k];
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) s_red[wave][k] = v;
  }
  __syncthreads();
  if (threadIdx.x < 12) {
    double t = 0;
    for (int q = 0; q < kGaussPerBlock / 64; ++q) t += s_red[q][threadIdx.x];
    W.pose_part[(int64_t)blockIdx.x * 16 + threadIdx.x] = t;
  }
}

// One workgroup per session: fixed-order sum of its block partials into the
// view-matrix gradient, and the pose (left-perturbation) gradient from it.
__global__ __launch_bounds__(256) void k_pose_reduce(Batch B, WsPtrs W) {
  __shared__ double s_acc[256][12];
  const SessionDev& S = session_of(B, blockIdx.x);
  const int b0 = S.block_base;
  const int b1 = (blockIdx.x + 1 < (unsigned)B.n_sessions)
                     ? session_of(B, blockIdx.x + 1).block_base
                     : B.b_total;
  double acc[12] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int b = b0 + (int)threadIdx.x; b < b1; b += 256)
    for (int k = 0; k < 12; ++k) acc[k] += W.pose_part[(int64_t)b * 16 + k];
  for (int k = 0; k < 12; ++k) s_acc[threadIdx.x][k] = acc[k];
  __syncthreads();
  for (int off = 128; off >= 1; off >>= 1) {
    if ((int)threadIdx.x < off)
      for (int k = 0; k < 12; ++k) s_acc[threadIdx.x][k] += s_acc[threadIdx.x + off][k];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double* g = s_acc[0];        // dL/dW row-major (9), dL/dt (3)
    if (S.g_viewmat)
      for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) S.g_viewmat[4 * i + j] = (float)g[3 * i + j];
        S.g_viewmat[4 * i + 3] = (float)g[9 + i];
      }
    if (S.g_pose6) {
      double vm[12];
      for (int k = 0; k < 12; ++k) vm[k] = S.viewmat[k];
      double A[9];                     // A = dL/dW W^T + dL/dt t^T
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
          A[3 * i + j] = g[3 * i] * vm[4 * j] + g[3 * i + 1] * vm[4 * j + 1] +
                         g[3 * i + 2] * vm[4 * j + 2] + g[9 + i] * vm[4 * j + 3];
      S.g_pose6[0] = (float)g[9];
      S.g_pose6[1] = (float)g[10];
      S.g_pose6[2] = (float)g[11];
      S.g_pose6[3] = (float)(A[7] - A[5]);
      S.g_pose6[4] = (float)(A[2] - A[6]);
      S.g_pose6[5] = (float)(A[3] - A[1]);
    }
  }
}

}  // namespace

template <int NV, bool ADAM>
static void gauss_bwd(const Batch& b, const WsPtrs& w, int grad_flags, hipStream_t st) {
  if (b.n_sessions == 1)
    k_gauss_bwd<NV, ADAM, true><<<b.b_total, kGaussPerBlock, 0, st>>>(b, w, grad_flags);
  else
    k_gauss_bwd<NV, ADAM, false><<<b.b_total, kGaussPerBlock, 0, st>>>(b, w, grad_flags);
}

hipError_t launch_preprocess_bwd(const Batch& b, const WsPtrs& w, int grad_flags, hipStream_t st,
                                 StageTimer* tm) {
  if (b.n_total > 0) {
    Scope sc(tm, kStMerge, st);
    const int grid = (b.n_total + kMergePerBlock - 1) / kMergePerBlock;
    if (grad_flags & RTGS_GRAD_MAP)
      k_merge<10><<<grid, 256, 0, st>>>(b, w);
    else
      k_merge<6><<<grid, 256, 0, st>>>(b, w);
  }
  if (b.b_total > 0) {
    Scope sc(tm, kStPreprocessBwd, st);
    if (grad_flags & RTGS_GRAD_ADAM)
      gauss_bwd<10, true>(b, w, grad_flags, st);
    else if (grad_flags & RTGS_GRAD_MAP)
      gauss_bwd<10, false>(b, w, grad_flags, st);
    else
      gauss_bwd<6, false>(b, w, grad_flags, st);
  }
  if ((grad_flags & RTGS_GRAD_POSE) && b.n_sessions > 0) {
    Scope sc(tm, kStPoseReduce, st);
    k_pose_reduce<<<b.n_sessions, 256, 0, st>>>(b, w);
  }
  return hipGetLastError();
}

}  // namespace rtgs
