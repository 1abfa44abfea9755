// gs_project kernel: EWA projection of 3D Gaussians and their SH colour.
//
// Sec. "Differentiable 3D Gaussian Splatting" of arXiv 2503.14171: a 3D
// Gaussian (mean mu, covariance Sigma from scale and rotation, opacity sigma,
// SH colour coefficients) projects to a 2D Gaussian with covariance
// Sigma' = J W Sigma W^T J^T, J the Jacobian of the local affine
// approximation of the perspective map.
//
// One thread per Gaussian.  The geometry is evaluated in FP64: MI355X runs
// FP64 vector FMAs at the FP32 rate and the kernel is bound by HBM traffic
// (236 B/Gaussian at SH degree 3), so the extra precision costs little; it
// keeps the FP32-stored conic and the FP64-stored mean accurate to the last
// bit, which the derivative buffers need (their sensitivity to the mean grows
// as 1/sigma_px^3).  The SH colour, which does not depend on the pixel, is
// summed in FP32.
#include <cmath>

#include "gsup_internal.h"

namespace gsup {
namespace {

// Widening of the exact alpha_min support box, in pixels, so that FP32
// rounding in the rasterizer's alpha test can never reach outside the tiles.
constexpr double kRectMargin = 0.25;
// The Jacobian is evaluated at the mean with its direction clamped to this
// multiple of the half field of view (keeps off-screen footprints finite).
constexpr double kFrustumClamp = 1.3;

// Camera of one view of a batch.
struct ProjView {
  int32_t width, height;
  double fx, fy, cx, cy;
  double V[12];
  double cam[3];
  double near_plane, far_plane;  // far_plane 0: none
  double limx, limy;
};

struct ProjParams {
  int64_t n;  // Gaussians (per view)
  int32_t nv, tile;
  double dilation;
  double alpha_min, log_alpha_min;
  ProjView view[GS_MAX_VIEWS];
};

// Real orthonormal SH basis (graphics sign convention, Condon-Shortley phase
// kept), ordered l^2 + l + m, evaluated as polynomials of the unit direction.
// Constants: K0 = 1/(2 sqrt(pi)); K1 = sqrt(3/(4 pi)); K2a = sqrt(15/pi)/2,
// K2b = sqrt(5/pi)/4, K2c = sqrt(15/pi)/4; K3a = sqrt(35/(2 pi))/4,
// K3b = sqrt(105/pi)/2, K3c = sqrt(21/(2 pi))/4, K3d = sqrt(7/pi)/4,
// K3e = sqrt(105/pi)/4.
template <int DEG>
__device__ __forceinline__ void sh_eval(float x, float y, float z, float* Y) {
  const float K0 = 0.28209479177387814f, K1 = 0.4886025119029199f;
  const float K2a = 1.0925484305920792f, K2b = 0.31539156525252005f, K2c = 0.5462742152960396f;
  const float K3a = 0.5900435899266435f, K3b = 2.890611442640554f, K3c = 0.4570457994644658f,
              K3d = 0.3731763325901154f, K3e = 1.445305721320277f;
  Y[0] = K0;
  if (DEG < 1) return;
  Y[1] = -K1 * y;
  Y[2] = K1 * z;
  Y[3] = -K1 * x;
  if (DEG < 2) return;
  const float xx = x * x, yy = y * y, zz = z * z;
  Y[4] = K2a * x * y;
  Y[5] = -K2a * y * z;
  Y[6] = K2b * (2.f * zz - xx - yy);
  Y[7] = -K2a * x * z;
  Y[8] = K2c * (xx - yy);
  if (DEG < 3) return;
  Y[9] = -K3a * y * (3.f * xx - yy);
  Y[10] = K3b * x * y * z;
  Y[11] = -K3c * y * (4.f * zz - xx - yy);
  Y[12] = K3d * z * (2.f * zz - 3.f * xx - 3.f * yy);
  Y[13] = -K3c * x * (4.f * zz - xx - yy);
  Y[14] = K3e * z * (xx - yy);
  Y[15] = -K3a * x * (xx - 3.f * yy);
}

template <int DEG, bool MULTI>
__global__ __launch_bounds__(256) void project_kernel(ProjParams p, const float* __restrict__ means,
                                                      const float* __restrict__ log_scales,
                                                      const float* __restrict__ quats,
                                                      const float* __restrict__ opacity,
                                                      const float* __restrict__ sh,
                                                      gs_splat* __restrict__ splats,
                                                      float* __restrict__ depth_out,
                                                      short4* __restrict__ rect_out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= p.n) return;
  constexpr int nb = (DEG + 1) * (DEG + 1);

  // the Gaussian's parameters are read once for all views of a batch (the
  // SH coefficients, read per view when on screen, come from the cache after
  // the first view)
  const double mu0 = means[3 * i], mu1 = means[3 * i + 1], mu2 = means[3 * i + 2];
  const double ls0 = log_scales[3 * i], ls1 = log_scales[3 * i + 1], ls2 = log_scales[3 * i + 2];
  const float4 q4 = reinterpret_cast<const float4*>(quats)[i];
  const float sig = opacity[i];

  const bool finite_in = isfinite(sig) && isfinite(mu0) && isfinite(mu1) && isfinite(mu2) &&
                         isfinite(ls0) && isfinite(ls1) && isfinite(ls2) && isfinite(q4.x) &&
                         isfinite(q4.y) && isfinite(q4.z) && isfinite(q4.w);

  const int nv = MULTI ? p.nv : 1;  // one view: a single, fully specialised pass
  for (int vi = 0; vi < nv; ++vi) {
  const ProjView& cv = p.view[vi];
  const int64_t o = (int64_t)vi * p.n + i;  // output record
  bool ok = finite_in;
  const double* V = cv.V;
  // camera-space position, summed left to right (products of FP32 values are
  // exact in FP64, so the depth is the correctly ordered sum)
  const double t0 = ((V[0] * mu0 + V[1] * mu1) + V[2] * mu2) + V[3];
  const double t1 = ((V[4] * mu0 + V[5] * mu1) + V[6] * mu2) + V[7];
  const double t2 = ((V[8] * mu0 + V[9] * mu1) + V[10] * mu2) + V[11];
  const double qn2 = (double)q4.x * q4.x + (double)q4.y * q4.y + (double)q4.z * q4.z +
                     (double)q4.w * q4.w;
  ok = ok && (t2 > cv.near_plane) && (cv.far_plane <= 0.0 || t2 <= cv.far_plane) && (qn2 > 0.0) &&
       ((double)sig >= p.alpha_min);

  float4 w0 = make_float4(0.f, 0.f, 0.f, 0.f), w1 = w0;
  double2 m2 = make_double2(0.0, 0.0);
  int4 rect = make_int4(0, 0, 0, 0);
  float dep = INFINITY;

  if (ok) {
    // rotation of the unit quaternion (w, x, y, z)
    const double qi = 1.0 / sqrt(qn2);
    const double w = q4.x * qi, x = q4.y * qi, y = q4.z * qi, z = q4.w * qi;
    double R[3][3] = {{1.0 - 2.0 * (y * y + z * z), 2.0 * (x * y - w * z), 2.0 * (x * z + w * y)},
                      {2.0 * (x * y + w * z), 1.0 - 2.0 * (x * x + z * z), 2.0 * (y * z - w * x)},
                      {2.0 * (x * z - w * y), 2.0 * (y * z + w * x), 1.0 - 2.0 * (x * x + y * y)}};
    const double s2[3] = {exp(2.0 * ls0), exp(2.0 * ls1), exp(2.0 * ls2)};
    // M = J W (2x3); Sigma' = M R S^2 R^T M^T = (M R) S^2 (M R)^T
    const double tz = t2, itz = 1.0 / t2;
    const double ux = fmin(cv.limx, fmax(-cv.limx, t0 * itz)) * tz;
    const double uy = fmin(cv.limy, fmax(-cv.limy, t1 * itz)) * tz;
    const double j00 = cv.fx * itz, j02 = -cv.fx * ux * itz * itz;
    const double j11 = cv.fy * itz, j12 = -cv.fy * uy * itz * itz;
    double M[2][3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      M[0][c] = j00 * V[c] + j02 * V[8 + c];
      M[1][c] = j11 * V[4 + c] + j12 * V[8 + c];
    }
    double P[2][3];  // P = M R
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) P[r][c] = M[r][0] * R[0][c] + M[r][1] * R[1][c] + M[r][2] * R[2][c];
    double sxx = p.dilation, sxy = 0.0, syy = p.dilation;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      sxx += P[0][k] * P[0][k] * s2[k];
      sxy += P[0][k] * P[1][k] * s2[k];
      syy += P[1][k] * P[1][k] * s2[k];
    }
    const double det = sxx * syy - sxy * sxy;
    if (det > 0.0) {
      const double mx = cv.fx * t0 * itz + cv.cx;
      const double my = cv.fy * t1 * itz + cv.cy;
      const double L = log((double)sig) - p.log_alpha_min;
      const double rx = sqrt(2.0 * L * sxx), ry = sqrt(2.0 * L * syy);
      double x0 = ceil(mx - rx - kRectMargin), x1 = floor(mx + rx + kRectMargin);
      double y0 = ceil(my - ry - kRectMargin), y1 = floor(my + ry + kRectMargin);
      x0 = fmax(x0, 0.0);
      y0 = fmax(y0, 0.0);
      x1 = fmin(x1, (double)(cv.width - 1));
      y1 = fmin(y1, (double)(cv.height - 1));
      if (x0 <= x1 && y0 <= y1) {
        // On screen: only now read the SH coefficients (3 nb floats), so the
        // splats that reach no tile cost no colour traffic.
        float coef[3 * nb];
        const float* shg = sh + (int64_t)3 * nb * i;
        if constexpr ((3 * nb) % 4 == 0) {
          const float4* s4 = reinterpret_cast<const float4*>(shg);
#pragma unroll
          for (int k = 0; k < 3 * nb / 4; ++k) {
            const float4 v = s4[k];
            coef[4 * k] = v.x;
            coef[4 * k + 1] = v.y;
            coef[4 * k + 2] = v.z;
            coef[4 * k + 3] = v.w;
          }
        } else {
#pragma unroll
          for (int k = 0; k < 3 * nb; ++k) coef[k] = shg[k];
        }
        bool fin = true;
#pragma unroll
        for (int k = 0; k < 3 * nb; ++k) fin = fin && isfinite(coef[k]);
        if (fin) {
          // view-dependent colour
          double dx = mu0 - cv.cam[0], dy = mu1 - cv.cam[1], dz = mu2 - cv.cam[2];
          const double dn2 = dx * dx + dy * dy + dz * dz;
          if (dn2 > 0.0) {
            const double idn = 1.0 / sqrt(dn2);
            dx *= idn;
            dy *= idn;
            dz *= idn;
          } else {
            dx = 0.0;
            dy = 0.0;
            dz = 1.0;
          }
          float Y[nb];
          sh_eval<DEG>((float)dx, (float)dy, (float)dz, Y);
          float col[3] = {0.f, 0.f, 0.f};
#pragma unroll
          for (int k = 0; k < nb; ++k) {
            col[0] = fmaf(Y[k], coef[3 * k], col[0]);
            col[1] = fmaf(Y[k], coef[3 * k + 1], col[1]);
            col[2] = fmaf(Y[k], coef[3 * k + 2], col[2]);
          }
          const double id = 1.0 / det;
          rect = make_int4((int)x0 / p.tile, (int)y0 / p.tile, (int)x1 / p.tile + 1,
                           (int)y1 / p.tile + 1);
          m2 = make_double2(mx, my);
          w0 = make_float4((float)(syy * id), (float)(-sxy * id), (float)(sxx * id), sig);
          w1 = make_float4(fmaxf(col[0] + 0.5f, 0.f), fmaxf(col[1] + 0.5f, 0.f),
                           fmaxf(col[2] + 0.5f, 0.f), (float)(2.0 * L));
          dep = (float)t2;
        }
      }
    }
  }
  double2* sp = reinterpret_cast<double2*>(splats + o);
  sp[0] = m2;
  float4* sf = reinterpret_cast<float4*>(splats + o);
  sf[1] = w0;
  sf[2] = w1;
  depth_out[o] = dep;
  rect_out[o] = make_short4((short)rect.x, (short)rect.y, (short)rect.z, (short)rect.w);
  }
}

// Gradient of the SH colour sum_k Y_k(d) coef_k with respect to the unit
// direction d: derivatives of the basis polynomials above.
template <int DEG>
__device__ __forceinline__ void sh_grad(double x, double y, double z, const double* w, double& gx,
                                        double& gy, double& gz) {
  // w[k] = sum_ch g_ch coef_k[ch] (the colour adjoint folded in)
  const double K1 = 0.4886025119029199;
  const double K2a = 1.0925484305920792, K2b = 0.31539156525252005, K2c = 0.5462742152960396;
  const double K3a = 0.5900435899266435, K3b = 2.890611442640554, K3c = 0.4570457994644658,
               K3d = 0.3731763325901154, K3e = 1.445305721320277;
  gx = gy = gz = 0.0;
  if (DEG < 1) return;
  gy += -K1 * w[1];
  gz += K1 * w[2];
  gx += -K1 * w[3];
  if (DEG < 2) return;
  const double xx = x * x, yy = y * y, zz = z * z;
  gx += K2a * y * w[4];
  gy += K2a * x * w[4];
  gy += -K2a * z * w[5];
  gz += -K2a * y * w[5];
  gx += -2.0 * K2b * x * w[6];
  gy += -2.0 * K2b * y * w[6];
  gz += 4.0 * K2b * z * w[6];
  gx += -K2a * z * w[7];
  gz += -K2a * x * w[7];
  gx += 2.0 * K2c * x * w[8];
  gy += -2.0 * K2c * y * w[8];
  if (DEG < 3) return;
  gx += -6.0 * K3a * x * y * w[9];
  gy += -3.0 * K3a * (xx - yy) * w[9];
  gx += K3b * y * z * w[10];
  gy += K3b * x * z * w[10];
  gz += K3b * x * y * w[10];
  gx += 2.0 * K3c * x * y * w[11];
  gy += -K3c * (4.0 * zz - xx - 3.0 * yy) * w[11];
  gz += -8.0 * K3c * y * z * w[11];
  gx += -6.0 * K3d * x * z * w[12];
  gy += -6.0 * K3d * y * z * w[12];
  gz += K3d * (6.0 * zz - 3.0 * xx - 3.0 * yy) * w[12];
  gx += -K3c * (4.0 * zz - 3.0 * xx - yy) * w[13];
  gy += 2.0 * K3c * x * y * w[13];
  gz += -8.0 * K3c * x * z * w[13];
  gx += 2.0 * K3e * x * z * w[14];
  gy += -2.0 * K3e * y * z * w[14];
  gz += K3e * (xx - yy) * w[14];
  gx += -3.0 * K3a * (xx - yy) * w[15];
  gy += 6.0 * K3a * x * y * w[15];
}

// Backward of the projection: dL/d(mean2d, conic, opacity, rgb) of every
// (view, Gaussian) record -> dL/d(means, log_scales, quats, opacity, sh),
// summed over the views.  One thread per Gaussian; the forward geometry is
// recomputed in FP64 and the chain rule applied step by step:
//   conic Q = Sigma'^-1:  dL/dSigma' = -Q (dL/dQ) Q  (dL/dQ symmetric, b counted twice)
//   Sigma' = P S^2 P^T + dilation I, P = M R, M = J W:
//     dL/dP = 2 dL/dSigma' P S^2, dL/ds_k^2 = (P^T dL/dSigma' P)_kk,
//     dL/dR = M^T dL/dP, dL/dM = dL/dP R^T, dL/dJ = dL/dM W^T
//   J(t) with the frustum-clamped direction, mean2d(t), t = W mu + t_W;
//   R(q / |q|); colour max(0, sum Y_k(d) k + 1/2), d = (mu - cam) / |mu - cam|.
template <int DEG>
__global__ __launch_bounds__(256) void project_bwd_kernel(
    ProjParams p, const float* __restrict__ means, const float* __restrict__ log_scales,
    const float* __restrict__ quats, const float* __restrict__ opacity,
    const float* __restrict__ sh, const float* __restrict__ dsplat, float* __restrict__ d_means,
    float* __restrict__ d_ls, float* __restrict__ d_quats, float* __restrict__ d_opacity,
    float* __restrict__ d_sh) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= p.n) return;
  constexpr int nb = (DEG + 1) * (DEG + 1);
  const double mu[3] = {means[3 * i], means[3 * i + 1], means[3 * i + 2]};
  const double ls[3] = {log_scales[3 * i], log_scales[3 * i + 1], log_scales[3 * i + 2]};
  const float4 q4 = reinterpret_cast<const float4*>(quats)[i];
  const double qv[4] = {q4.x, q4.y, q4.z, q4.w};
  const double qn2 = qv[0] * qv[0] + qv[1] * qv[1] + qv[2] * qv[2] + qv[3] * qv[3];
  double gmu[3] = {0, 0, 0}, gls[3] = {0, 0, 0}, gq[4] = {0, 0, 0, 0}, gsig = 0.0;
  float gsh[3 * nb];  // FP32 accumulation over at most 16 views
#pragma unroll
  for (int k = 0; k < 3 * nb; ++k) gsh[k] = 0.f;
  const double qi = qn2 > 0.0 ? 1.0 / sqrt(qn2) : 0.0;
  const double w = qv[0] * qi, x = qv[1] * qi, y = qv[2] * qi, z = qv[3] * qi;
  const double R[3][3] = {{1.0 - 2.0 * (y * y + z * z), 2.0 * (x * y - w * z), 2.0 * (x * z + w * y)},
                          {2.0 * (x * y + w * z), 1.0 - 2.0 * (x * x + z * z), 2.0 * (y * z - w * x)},
                          {2.0 * (x * z - w * y), 2.0 * (y * z + w * x), 1.0 - 2.0 * (x * x + y * y)}};
  const double s2[3] = {exp(2.0 * ls[0]), exp(2.0 * ls[1]), exp(2.0 * ls[2])};
  double gR[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};

  for (int vi = 0; vi < p.nv; ++vi) {
    const float* ds = dsplat + ((int64_t)vi * p.n + i) * 9;
    const float g_mx = ds[0], g_my = ds[1], g_a = ds[2], g_b = ds[3], g_c = ds[4];
    const float g_sig = ds[5], g_r = ds[6], g_g = ds[7], g_bl = ds[8];
    if (g_mx == 0.f && g_my == 0.f && g_a == 0.f && g_b == 0.f && g_c == 0.f && g_sig == 0.f &&
        g_r == 0.f && g_g == 0.f && g_bl == 0.f)
      continue;  // never rasterized in this view (culled records have no gradient)
    const ProjView& cv = p.view[vi];
    const double* V = cv.V;
    const double t0 = ((V[0] * mu[0] + V[1] * mu[1]) + V[2] * mu[2]) + V[3];
    const double t1 = ((V[4] * mu[0] + V[5] * mu[1]) + V[6] * mu[2]) + V[7];
    const double t2 = ((V[8] * mu[0] + V[9] * mu[1]) + V[10] * mu[2]) + V[11];
    const double itz = 1.0 / t2;
    const double rx0 = t0 * itz, ry0 = t1 * itz;
    const double rx = fmin(cv.limx, fmax(-cv.limx, rx0));
    const double ry = fmin(cv.limy, fmax(-cv.limy, ry0));
    const bool clx = rx != rx0, cly = ry != ry0;
    const double j00 = cv.fx * itz, j02 = -cv.fx * rx * itz;
    const double j11 = cv.fy * itz, j12 = -cv.fy * ry * itz;
    double M[2][3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      M[0][c] = j00 * V[c] + j02 * V[8 + c];
      M[1][c] = j11 * V[4 + c] + j12 * V[8 + c];
    }
    double P[2][3];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) P[r][c] = M[r][0] * R[0][c] + M[r][1] * R[1][c] + M[r][2] * R[2][c];
    double sxx = p.dilation, sxy = 0.0, syy = p.dilation;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      sxx += P[0][k] * P[0][k] * s2[k];
      sxy += P[0][k] * P[1][k] * s2[k];
      syy += P[1][k] * P[1][k] * s2[k];
    }
    const double det = sxx * syy - sxy * sxy;
    const double id = 1.0 / det;
    const double Qa = syy * id, Qb = -sxy * id, Qc = sxx * id;
    // dL/dSigma' = -Q G Q with G = [[g_a, g_b/2], [g_b/2, g_c]]
    const double G00 = g_a, G01 = 0.5 * g_b, G11 = g_c;
    const double QG00 = Qa * G00 + Qb * G01, QG01 = Qa * G01 + Qb * G11;
    const double QG10 = Qb * G00 + Qc * G01, QG11 = Qb * G01 + Qc * G11;
    const double D00 = -(QG00 * Qa + QG01 * Qb), D01 = -(QG00 * Qb + QG01 * Qc);
    const double D11 = -(QG10 * Qb + QG11 * Qc);
    double gP[2][3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      gP[0][k] = 2.0 * (D00 * P[0][k] + D01 * P[1][k]) * s2[k];
      gP[1][k] = 2.0 * (D01 * P[0][k] + D11 * P[1][k]) * s2[k];
      const double gs2 = P[0][k] * (D00 * P[0][k] + D01 * P[1][k]) +
                         P[1][k] * (D01 * P[0][k] + D11 * P[1][k]);
      gls[k] += gs2 * 2.0 * s2[k];
    }
    // dL/dR = M^T gP, dL/dM = gP R^T
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) gR[r][c] += M[0][r] * gP[0][c] + M[1][r] * gP[1][c];
    double gM[2][3];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) gM[r][c] = gP[r][0] * R[c][0] + gP[r][1] * R[c][1] + gP[r][2] * R[c][2];
    // dL/dJ for the four non-zero entries (M_r. = sum_c J_rc W_c.)
    const double gJ00 = gM[0][0] * V[0] + gM[0][1] * V[1] + gM[0][2] * V[2];
    const double gJ02 = gM[0][0] * V[8] + gM[0][1] * V[9] + gM[0][2] * V[10];
    const double gJ11 = gM[1][0] * V[4] + gM[1][1] * V[5] + gM[1][2] * V[6];
    const double gJ12 = gM[1][0] * V[8] + gM[1][1] * V[9] + gM[1][2] * V[10];
    const double itz2 = itz * itz;
    double gt0 = 0.0, gt1 = 0.0, gt2 = 0.0;
    gt2 += -cv.fx * itz2 * gJ00 - cv.fy * itz2 * gJ11;
    // j02 = -fx rx / t2 with rx = t0 / t2 unless clamped
    if (clx) {
      gt2 += cv.fx * rx * itz2 * gJ02;
    } else {
      gt0 += -cv.fx * itz2 * gJ02;
      gt2 += 2.0 * cv.fx * t0 * itz2 * itz * gJ02;
    }
    if (cly) {
      gt2 += cv.fy * ry * itz2 * gJ12;
    } else {
      gt1 += -cv.fy * itz2 * gJ12;
      gt2 += 2.0 * cv.fy * t1 * itz2 * itz * gJ12;
    }
    // mean2d = (fx t0 / t2 + cx, fy t1 / t2 + cy)
    gt0 += cv.fx * itz * g_mx;
    gt1 += cv.fy * itz * g_my;
    gt2 += -(cv.fx * t0 * g_mx + cv.fy * t1 * g_my) * itz2;
#pragma unroll
    for (int c = 0; c < 3; ++c) gmu[c] += V[c] * gt0 + V[4 + c] * gt1 + V[8 + c] * gt2;
    gsig += g_sig;
    // colour: max(0, s + 1/2) per channel, s = sum_k Y_k(d) coef_k
    double dx = mu[0] - cv.cam[0], dy = mu[1] - cv.cam[1], dz = mu[2] - cv.cam[2];
    const double dn2 = dx * dx + dy * dy + dz * dz;
    const double idn = dn2 > 0.0 ? 1.0 / sqrt(dn2) : 0.0;
    if (dn2 > 0.0) {
      dx *= idn;
      dy *= idn;
      dz *= idn;
    } else {
      dx = 0.0;
      dy = 0.0;
      dz = 1.0;
    }
    float Y[nb];
    sh_eval<DEG>((float)dx, (float)dy, (float)dz, Y);
    const float* shg = sh + (int64_t)3 * nb * i;
    float gch[3] = {g_r, g_g, g_bl};
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
      float col = 0.f;
#pragma unroll
      for (int k = 0; k < nb; ++k) col = fmaf(Y[k], shg[3 * k + ch], col);
      if (!(col + 0.5f > 0.f)) gch[ch] = 0.f;  // clamped at zero
    }
    double wk[nb];
#pragma unroll
    for (int k = 0; k < nb; ++k) {
      wk[k] = (double)gch[0] * shg[3 * k] + (double)gch[1] * shg[3 * k + 1] +
              (double)gch[2] * shg[3 * k + 2];
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) gsh[3 * k + ch] = fmaf(Y[k], gch[ch], gsh[3 * k + ch]);
    }
    if (dn2 > 0.0) {
      double gdx, gdy, gdz;
      sh_grad<DEG>(dx, dy, dz, wk, gdx, gdy, gdz);
      // d = v / |v|: dL/dv = (g - d (d . g)) / |v|
      const double dg = dx * gdx + dy * gdy + dz * gdz;
      gmu[0] += (gdx - dx * dg) * idn;
      gmu[1] += (gdy - dy * dg) * idn;
      gmu[2] += (gdz - dz * dg) * idn;
    }
  }
  // quaternion: dL/dq-hat from dL/dR, then the normalisation
  double gqh[4];
  gqh[0] = 2.0 * (-z * gR[0][1] + y * gR[0][2] + z * gR[1][0] - x * gR[1][2] - y * gR[2][0] + x * gR[2][1]);
  gqh[1] = 2.0 * (y * gR[0][1] + z * gR[0][2] + y * gR[1][0] - 2.0 * x * gR[1][1] - w * gR[1][2] +
                  z * gR[2][0] + w * gR[2][1] - 2.0 * x * gR[2][2]);
  gqh[2] = 2.0 * (-2.0 * y * gR[0][0] + x * gR[0][1] + w * gR[0][2] + x * gR[1][0] + z * gR[1][2] -
                  w * gR[2][0] + z * gR[2][1] - 2.0 * y * gR[2][2]);
  gqh[3] = 2.0 * (-2.0 * z * gR[0][0] - w * gR[0][1] + x * gR[0][2] + w * gR[1][0] -
                  2.0 * z * gR[1][1] + y * gR[1][2] + x * gR[2][0] + y * gR[2][1]);
  const double qh[4] = {w, x, y, z};
  const double dq = qh[0] * gqh[0] + qh[1] * gqh[1] + qh[2] * gqh[2] + qh[3] * gqh[3];
#pragma unroll
  for (int k = 0; k < 4; ++k) gq[k] = (gqh[k] - qh[k] * dq) * qi;
  for (int c = 0; c < 3; ++c) {
    d_means[3 * i + c] = (float)gmu[c];
    d_ls[3 * i + c] = (float)gls[c];
  }
  reinterpret_cast<float4*>(d_quats)[i] =
      make_float4((float)gq[0], (float)gq[1], (float)gq[2], (float)gq[3]);
  d_opacity[i] = (float)gsig;
  float* gs = d_sh + (int64_t)3 * nb * i;
#pragma unroll
  for (int k = 0; k < 3 * nb; ++k) gs[k] = gsh[k];
}

ProjParams make_proj_params(int64_t n, int32_t nv, const gs_camera* cams,
                            const gs_raster_cfg& cfg) {
  ProjParams p{};
  p.n = n;
  p.nv = nv;
  p.tile = cfg.tile_size;
  p.dilation = cfg.dilation;
  p.alpha_min = cfg.alpha_min;
  p.log_alpha_min = log((double)cfg.alpha_min);
  for (int v = 0; v < nv; ++v) {
    const gs_camera& cam = cams[v];
    ProjView& c = p.view[v];
    c.width = cam.width;
    c.height = cam.height;
    c.fx = cam.fx;
    c.fy = cam.fy;
    c.cx = cam.cx;
    c.cy = cam.cy;
    for (int k = 0; k < 12; ++k) c.V[k] = cam.view[k];
    for (int k = 0; k < 3; ++k) c.cam[k] = cam.cam_pos[k];
    c.near_plane = cam.near_plane;
    c.far_plane = cam.far_plane;
    c.limx = kFrustumClamp * (0.5 * cam.width) / (double)cam.fx;
    c.limy = kFrustumClamp * (0.5 * cam.height) / (double)cam.fy;
  }
  return p;
}

}  // namespace

hipError_t launch_project(int64_t n, const float* means, const float* log_scales,
                          const float* quats, const float* opacity, const float* sh, int32_t nv,
                          const gs_camera* cams, const gs_raster_cfg& cfg, gs_splat* splats,
                          float* depth, int16_t* rect, hipStream_t stream) {
  const ProjParams p = make_proj_params(n, nv, cams, cfg);
  const int threads = 256;
  const int64_t blocks = ceil_div(n, threads);
  short4* r4 = reinterpret_cast<short4*>(rect);
  const dim3 g((unsigned)blocks), b(threads);
#define GS_PROJ(D)                                                                              \
  if (nv > 1)                                                                                   \
    project_kernel<D, true><<<g, b, 0, stream>>>(p, means, log_scales, quats, opacity, sh,     \
                                                 splats, depth, r4);                            \
  else                                                                                          \
    project_kernel<D, false><<<g, b, 0, stream>>>(p, means, log_scales, quats, opacity, sh,    \
                                                  splats, depth, r4);
  switch (cfg.sh_degree) {
    case 0: GS_PROJ(0) break;
    case 1: GS_PROJ(1) break;
    case 2: GS_PROJ(2) break;
    default: GS_PROJ(3) break;
  }
#undef GS_PROJ
  return hipGetLastError();
}

hipError_t launch_project_backward(int64_t n, const float* means, const float* log_scales,
                                   const float* quats, const float* opacity, const float* sh,
                                   int32_t nv, const gs_camera* cams, const gs_raster_cfg& cfg,
                                   const float* dsplat, float* d_means, float* d_log_scales,
                                   float* d_quats, float* d_opacity, float* d_sh,
                                   hipStream_t stream) {
  const ProjParams p = make_proj_params(n, nv, cams, cfg);
  const dim3 g((unsigned)ceil_div(n, 256)), b(256);
  switch (cfg.sh_degree) {
    case 0: project_bwd_kernel<0><<<g, b, 0, stream>>>(p, means, log_scales, quats, opacity, sh, dsplat, d_means, d_log_scales, d_quats, d_opacity, d_sh); break;
    case 1: project_bwd_kernel<1><<<g, b, 0, stream>>>(p, means, log_scales, quats, opacity, sh, dsplat, d_means, d_log_scales, d_quats, d_opacity, d_sh); break;
    case 2: project_bwd_kernel<2><<<g, b, 0, stream>>>(p, means, log_scales, quats, opacity, sh, dsplat, d_means, d_log_scales, d_quats, d_opacity, d_sh); break;
    default: project_bwd_kernel<3><<<g, b, 0, stream>>>(p, means, log_scales, quats, opacity, sh, dsplat, d_means, d_log_scales, d_quats, d_opacity, d_sh); break;
  }
  return hipGetLastError();
}

}  // namespace gsup
