// Pose update of the tracking stage (Sec. 3.1: tracking updates the camera
// pose from dL/dP, Step 5): Adam on the left-perturbation tangent
// xi = (rho, phi) at xi = 0, then re-linearisation T <- Exp(-step) T so the
// tangent returns to zero.  One thread per session, float64 arithmetic; the
// view matrix stays on the device.
#include "rtgs_internal.h"

namespace rtgs {
namespace {

static_assert(sizeof(PoseArgs) <= 4000, "pose update table must fit the kernel arguments");

// Exp of xi = (rho, phi) as R (3x3) and t = V rho, with the series of
// sin t / t, (1 - cos t) / t^2, (t - sin t) / t^3 near zero.
__device__ void se3_exp(const double* xi, double* R, double* t) {
  const double px = xi[3], py = xi[4], pz = xi[5];
  const double th2 = px * px + py * py + pz * pz;
  double a, b, c;
  if (th2 < 1e-8) {
    a = 1.0 - th2 / 6.0 + th2 * th2 / 120.0;
    b = 0.5 - th2 / 24.0 + th2 * th2 / 720.0;
    c = 1.0 / 6.0 - th2 / 120.0 + th2 * th2 / 5040.0;
  } else {
    const double th = sqrt(th2);
    a = sin(th) / th;
    b = (1.0 - cos(th)) / th2;
    c = (th - sin(th)) / (th2 * th);
  }
  // W = [phi]_x, W^2 = phi phi^T - th2 I
  const double W[9] = {0.0, -pz, py, pz, 0.0, -px, -py, px, 0.0};
  const double P[3] = {px, py, pz};
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      const double w2 = P[i] * P[j] - (i == j ? th2 : 0.0);
      const double e = i == j ? 1.0 : 0.0;
      R[3 * i + j] = e + a * W[3 * i + j] + b * w2;
    }
  for (int i = 0; i < 3; ++i) {
    double s = 0.0;
    for (int j = 0; j < 3; ++j) {
      const double w2 = P[i] * P[j] - (i == j ? th2 : 0.0);
      const double e = i == j ? 1.0 : 0.0;
      s += (e + b * W[3 * i + j] + c * w2) * xi[j];
    }
    t[i] = s;
  }
}

__global__ void k_pose_update(PoseArgs a) {
  const int s = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (s >= a.n) return;
  const PoseItemDev& it = a.item[s];
  double step[6];
  for (int i = 0; i < 6; ++i) {
    const double g = it.g_pose6[i];
    const double m = a.beta1 * (double)it.exp_avg[i] + (1.0 - a.beta1) * g;
    const double v = a.beta2 * (double)it.exp_avg_sq[i] + (1.0 - a.beta2) * g * g;
    it.exp_avg[i] = (float)m;
    it.exp_avg_sq[i] = (float)v;
    const double lr = i < 3 ? it.lr_rho : it.lr_phi;
    // descent step on xi, applied as T <- Exp(-step) T
    step[i] = -lr * (m / it.bc1) / (sqrt(v / it.bc2) + a.eps);
  }
  double R[9], t[3], T[12];
  se3_exp(step, R, t);
  for (int k = 0; k < 12; ++k) T[k] = it.viewmat[k];
  for (int i = 0; i < 3; ++i) {
    for (int j = 0; j < 4; ++j) {
      double s2 = j == 3 ? t[i] : 0.0;
      for (int k = 0; k < 3; ++k) s2 += R[3 * i + k] * T[4 * k + j];
      it.viewmat[4 * i + j] = (float)s2;
    }
  }
}

}  // namespace

hipError_t launch_pose_update(const PoseArgs& a, hipStream_t st) {
  if (a.n <= 0) return hipSuccess;
  k_pose_update<<<(a.n + 63) / 64, 64, 0, st>>>(a);
  return hipGetLastError();
}

}  // namespace rtgs
