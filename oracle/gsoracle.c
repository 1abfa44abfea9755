/*
 * gsoracle.c -- plain FP64 CPU oracle for gradient-aware upscaling of 3D
 * Gaussian Splatting images (Niedermayr, Neuhauser, Westermann: "Lightweight
 * Gradient-Aware Upscaling of 3D Gaussian Splatting Images", arXiv 2503.14171).
 *
 * TEST INFRASTRUCTURE.  This library exists to check the HIP implementation.
 * Only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark load it; the product path never does.  It shares no code, header,
 * constant or helper with the HIP implementation.
 *
 * Everything is evaluated in double precision from the FP32 scene values.
 * Nothing is blocked, tiled or fused: every image point is composited by a
 * walk over the whole depth-sorted Gaussian list, exactly as the blending
 * equations are written.  The functions and the passages they follow:
 *
 *   or_sh_basis      real spherical harmonics of degree <= 3 (Sec. "Differentiable
 *                    3D Gaussian Splatting": SH colour), from the associated
 *                    Legendre definition with the Condon-Shortley phase.
 *   or_project       covariance from scale and rotation, view transform, EWA
 *                    projection Sigma' = J W Sigma W^T J^T (Sec. "Differentiable
 *                    3D Gaussian Splatting", projection equation), low-pass
 *                    dilation, conic, SH colour, depth, exact alpha_min support box.
 *   or_composite     front-to-back alpha blending with the analytical screen-space
 *                    derivatives dI/dx, dI/dy, d2I/dxdy (Suppl. "3DGS Gradient
 *                    Computation - Forward pass", recurrences for B_i, A_i and
 *                    their x, y and xy derivatives), plus near-tie analysis.
 *   or_patch_eval    bicubic patch p(x,y) = [1 x x^2 x^3] A [1 y y^2 y^3]^T with
 *                    A = C^-1 F C^-T (Sec. "Image Gradient Based Upscaling",
 *                    Suppl. "Spline Image Interpolation") and its derivatives.
 *   or_upscale       the same patch evaluated at every high-res pixel centre.
 *   or_upscale_adjoint  transpose of or_upscale: gradient of a loss with
 *                    respect to the low-res values and derivatives.
 *   or_composite_adjoint  gradient of a loss on (I, I_x, I_y, I_xy) with respect
 *                    to every Gaussian's 2D mean, conic, opacity and colour
 *                    (Suppl. "3DGS Gradient Computation - Backward pass":
 *                    back-to-front recurrences for B-hat and its derivatives,
 *                    dI/d alpha_k = T_k (c_k - B-hat_{k+1}) and its screen
 *                    derivatives, chain rule to the parameters; colour weights).
 *
 * Readings where the paper is silent or garbled (all shared with the HIP path
 * by specification, never by code):
 *   - Gaussian exponent g = -1/2 d^T Sigma'^-1 d with d = (x - mu_x, y - mu_y).
 *   - Sigma' gets a dilation (default 0.3 px^2) on its diagonal.
 *   - Fragments with alpha < alpha_min are skipped; alpha > alpha_max is clamped
 *     to alpha_max with zero screen derivatives; after blending a fragment the
 *     walk stops once the transmittance 1 - A falls below t_min.
 *   - Depth order is by camera z rounded to FP32, ties by Gaussian index
 *     (the caller supplies that order).
 *   - Pixel centres at integer coordinates; high-res pixel X samples the
 *     low-res coordinate u = (X + 1/2) w / W - 1/2; border cells extrapolate.
 *   - Colour = max(0, sum_lm Y_lm(d) k_lm + 1/2), d = normalize(mu - cam_pos).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_MAX_AMB 3   /* near-tie decisions enumerated per point (2^3 variants) */
#define OR_MAX_VAR 8

typedef struct {
  int32_t width, height;
  double fx, fy, cx, cy;
  double view[12];    /* row-major [R | t], world -> camera, OpenCV axes */
  double cam_pos[3];  /* camera centre in world space */
  double near_plane;
  double far_plane;   /* 0: none */
} or_camera;

typedef struct {
  int32_t sh_degree;
  double dilation;
  double alpha_min, alpha_max, t_min;
  double bg[3];
  double tie_alpha;   /* relative margin on alpha decisions that counts as a near tie */
  double tie_t;       /* relative margin on the transmittance stop decision */
} or_config;

/* ------------------------------------------------------------------------- */
/* Real spherical harmonics                                                  */
/* ------------------------------------------------------------------------- */

static double factorial(int k) {
  double r = 1.0;
  for (int i = 2; i <= k; ++i) r *= (double)i;
  return r;
}

/* Associated Legendre function P_l^m(x), m >= 0, with the Condon-Shortley
 * phase (-1)^m, by the textbook recurrences in l. */
static double assoc_legendre(int l, int m, double x) {
  double pmm = 1.0;
  double s = sqrt(fmax(0.0, 1.0 - x * x));
  for (int i = 1; i <= m; ++i) pmm *= -(2.0 * i - 1.0) * s;
  if (l == m) return pmm;
  double pmm1 = x * (2.0 * m + 1.0) * pmm;
  if (l == m + 1) return pmm1;
  double pll = 0.0;
  for (int ll = m + 2; ll <= l; ++ll) {
    pll = ((2.0 * ll - 1.0) * x * pmm1 - (ll + m - 1.0) * pmm) / (double)(ll - m);
    pmm = pmm1;
    pmm1 = pll;
  }
  return pll;
}

/* Real orthonormal SH at unit direction (x, y, z), ordered l^2 + l + m.
 * m > 0: sqrt2 K_lm P_l^m cos(m phi); m < 0: sqrt2 K_l|m| P_l^|m| sin(|m| phi);
 * m = 0: K_l0 P_l^0.  K_lm = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!). */
static void sh_basis(int deg, double x, double y, double z, double* out) {
  double ct = z;
  double phi = atan2(y, x);
  for (int l = 0; l <= deg; ++l) {
    for (int m = -l; m <= l; ++m) {
      int am = m < 0 ? -m : m;
      double K = sqrt((2.0 * l + 1.0) / (4.0 * M_PI) * factorial(l - am) / factorial(l + am));
      double P = assoc_legendre(l, am, ct);
      double v;
      if (m > 0) v = sqrt(2.0) * K * P * cos(am * phi);
      else if (m < 0) v = sqrt(2.0) * K * P * sin(am * phi);
      else v = K * P;
      out[l * l + l + m] = v;
    }
  }
}

void or_sh_basis(int32_t deg, int64_t n, const double* dirs, double* out) {
  int nb = (deg + 1) * (deg + 1);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    const double* d = dirs + 3 * i;
    double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    sh_basis(deg, d[0] / r, d[1] / r, d[2] / r, out + (int64_t)nb * i);
  }
}

/* ------------------------------------------------------------------------- */
/* Projection                                                                */
/* ------------------------------------------------------------------------- */

/* Rotation matrix of the unit quaternion (w, x, y, z). */
static void quat_to_rot(double w, double x, double y, double z, double R[3][3]) {
  R[0][0] = 1.0 - 2.0 * (y * y + z * z);
  R[0][1] = 2.0 * (x * y - w * z);
  R[0][2] = 2.0 * (x * z + w * y);
  R[1][0] = 2.0 * (x * y + w * z);
  R[1][1] = 1.0 - 2.0 * (x * x + z * z);
  R[1][2] = 2.0 * (y * z - w * x);
  R[2][0] = 2.0 * (x * z - w * y);
  R[2][1] = 2.0 * (y * z + w * x);
  R[2][2] = 1.0 - 2.0 * (x * x + y * y);
}

/* Per Gaussian i:
 *   valid[i]      1 if the Gaussian takes part in compositing
 *   mean2d[2i..]  image-plane mean (pixels)
 *   cov2d[3i..]   dilated 2D covariance (xx, xy, yy)
 *   conic[3i..]   its inverse (a, b, c) = [[a, b], [b, c]]
 *   opac[i]       opacity sigma (copied)
 *   rgb[3i..]     SH colour
 *   depth[i]      camera-space z
 *   bbox[4i..]    exact box of {alpha >= alpha_min}: xmin, xmax, ymin, ymax
 * A Gaussian is culled (valid = 0) when an input is not finite, when its
 * camera z is at or before the near plane, when the 2D covariance is not
 * positive definite, or when sigma < alpha_min (it can never reach alpha_min). */
void or_project(int64_t n, const double* means, const double* log_scales, const double* quats,
                const double* opacity, const double* sh, const or_camera* cam, const or_config* cfg,
                int32_t* valid, double* mean2d, double* cov2d, double* conic, double* opac,
                double* rgb, double* depth, double* bbox) {
  const int nb = (cfg->sh_degree + 1) * (cfg->sh_degree + 1);
  const double* V = cam->view;
  const double limx = 1.3 * (0.5 * cam->width) / cam->fx;
  const double limy = 1.3 * (0.5 * cam->height) / cam->fy;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    valid[i] = 0;
    mean2d[2 * i] = mean2d[2 * i + 1] = 0.0;
    for (int k = 0; k < 3; ++k) cov2d[3 * i + k] = conic[3 * i + k] = rgb[3 * i + k] = 0.0;
    for (int k = 0; k < 4; ++k) bbox[4 * i + k] = 0.0;
    depth[i] = 0.0;
    opac[i] = opacity[i];

    double mu[3] = {means[3 * i], means[3 * i + 1], means[3 * i + 2]};
    double ls[3] = {log_scales[3 * i], log_scales[3 * i + 1], log_scales[3 * i + 2]};
    double q[4] = {quats[4 * i], quats[4 * i + 1], quats[4 * i + 2], quats[4 * i + 3]};
    int finite = isfinite(opacity[i]);
    for (int k = 0; k < 3; ++k) finite = finite && isfinite(mu[k]) && isfinite(ls[k]);
    for (int k = 0; k < 4; ++k) finite = finite && isfinite(q[k]);
    for (int k = 0; k < 3 * nb; ++k) finite = finite && isfinite(sh[(int64_t)3 * nb * i + k]);
    if (!finite) continue;
    double qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    if (!(qn > 0.0)) continue;

    /* camera-space position t = W mu + t_W, summed left to right */
    double t[3];
    for (int r = 0; r < 3; ++r)
      t[r] = ((V[4 * r] * mu[0] + V[4 * r + 1] * mu[1]) + V[4 * r + 2] * mu[2]) + V[4 * r + 3];
    depth[i] = t[2];
    if (!(t[2] > cam->near_plane)) continue;
    if (cam->far_plane > 0.0 && t[2] > cam->far_plane) continue;

    /* world covariance Sigma = R S S^T R^T */
    double R[3][3];
    quat_to_rot(q[0] / qn, q[1] / qn, q[2] / qn, q[3] / qn, R);
    double s[3] = {exp(ls[0]), exp(ls[1]), exp(ls[2])};
    double Sig[3][3];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) {
        double acc = 0.0;
        for (int k = 0; k < 3; ++k) acc += R[r][k] * s[k] * s[k] * R[c][k];
        Sig[r][c] = acc;
      }

    /* Jacobian of the local affine approximation of the perspective map,
     * evaluated at the mean with its direction clamped to 1.3x the frustum. */
    double tz = t[2];
    double ux = fmin(limx, fmax(-limx, t[0] / tz)) * tz;
    double uy = fmin(limy, fmax(-limy, t[1] / tz)) * tz;
    double J[2][3] = {{cam->fx / tz, 0.0, -cam->fx * ux / (tz * tz)},
                      {0.0, cam->fy / tz, -cam->fy * uy / (tz * tz)}};
    /* T = J W, Sigma' = T Sigma T^T + dilation I */
    double T[2][3];
    for (int r = 0; r < 2; ++r)
      for (int c = 0; c < 3; ++c) {
        double acc = 0.0;
        for (int k = 0; k < 3; ++k) acc += J[r][k] * V[4 * k + c];
        T[r][c] = acc;
      }
    double S2[2][2];
    for (int r = 0; r < 2; ++r)
      for (int c = 0; c < 2; ++c) {
        double acc = 0.0;
        for (int k = 0; k < 3; ++k)
          for (int l = 0; l < 3; ++l) acc += T[r][k] * Sig[k][l] * T[c][l];
        S2[r][c] = acc;
      }
    S2[0][0] += cfg->dilation;
    S2[1][1] += cfg->dilation;
    double det = S2[0][0] * S2[1][1] - S2[0][1] * S2[1][0];
    if (!(det > 0.0)) continue;
    if (!(opacity[i] >= cfg->alpha_min)) continue;

    cov2d[3 * i] = S2[0][0];
    cov2d[3 * i + 1] = S2[0][1];
    cov2d[3 * i + 2] = S2[1][1];
    conic[3 * i] = S2[1][1] / det;
    conic[3 * i + 1] = -S2[0][1] / det;
    conic[3 * i + 2] = S2[0][0] / det;
    mean2d[2 * i] = cam->fx * t[0] / tz + cam->cx;
    mean2d[2 * i + 1] = cam->fy * t[1] / tz + cam->cy;

    /* {alpha >= alpha_min} = {d^T Q d <= 2L}, L = ln(sigma / alpha_min);
     * the box of that ellipse has half extents sqrt(2L Sigma'_xx), sqrt(2L Sigma'_yy). */
    double L = log(opacity[i] / cfg->alpha_min);
    double rx = sqrt(2.0 * L * S2[0][0]);
    double ry = sqrt(2.0 * L * S2[1][1]);
    bbox[4 * i] = mean2d[2 * i] - rx;
    bbox[4 * i + 1] = mean2d[2 * i] + rx;
    bbox[4 * i + 2] = mean2d[2 * i + 1] - ry;
    bbox[4 * i + 3] = mean2d[2 * i + 1] + ry;

    /* view-dependent colour */
    double dir[3] = {mu[0] - cam->cam_pos[0], mu[1] - cam->cam_pos[1], mu[2] - cam->cam_pos[2]};
    double dn = sqrt(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
    double Y[16];
    if (dn > 0.0) sh_basis(cfg->sh_degree, dir[0] / dn, dir[1] / dn, dir[2] / dn, Y);
    else sh_basis(cfg->sh_degree, 0.0, 0.0, 1.0, Y);
    for (int ch = 0; ch < 3; ++ch) {
      double acc = 0.0;
      for (int k = 0; k < nb; ++k) acc += Y[k] * (double)sh[(int64_t)3 * nb * i + 3 * k + ch];
      rgb[3 * i + ch] = fmax(0.0, acc + 0.5);
    }
    valid[i] = 1;
  }
}

/* ------------------------------------------------------------------------- */
/* Compositing with screen-space derivatives                                 */
/* ------------------------------------------------------------------------- */

enum { OR_DEC_SKIP = 0, OR_DEC_CLAMP = 1, OR_DEC_STOP = 2 };

typedef struct {
  int64_t pos;  /* position in the depth-ordered list */
  int kind;     /* OR_DEC_* */
} or_decision;

static void note_tie(or_decision* amb, int* namb, int cap, int64_t k, int kind) {
  if (!amb) return;
  if (*namb < cap) {
    amb[*namb].pos = k;
    amb[*namb].kind = kind;
  }
  ++*namb;
}

/* Outcome of decision `kind` at list position k: the plain comparison, inverted
 * when the caller asks for it and the comparison is a near tie (margin < tie). */
static int decide(int plain, double margin, double tie, const or_decision* flip, int nflip,
                  int64_t k, int kind, or_decision* amb, int* namb, int amb_cap) {
  int near = margin < tie;
  if (near) note_tie(amb, namb, amb_cap, k, kind);
  for (int f = 0; f < nflip; ++f)
    if (near && flip[f].pos == k && flip[f].kind == kind) return !plain;
  return plain;
}

/* One walk over the depth-ordered list at image point (x, y).
 * Near ties met on the way are appended to `amb` (up to amb_cap; *namb counts
 * all of them).  Returns the number of blended fragments. */
static int64_t walk(double x, double y, int64_t m, const int64_t* order, const double* mean2d,
                    const double* conic, const double* opac, const double* rgb,
                    const or_config* cfg, const or_decision* flip, int nflip, double out[12],
                    or_decision* amb, int* namb, int amb_cap) {
  double A = 0.0, Ax = 0.0, Ay = 0.0, Axy = 0.0;
  double B[3] = {0, 0, 0}, Bx[3] = {0, 0, 0}, By[3] = {0, 0, 0}, Bxy[3] = {0, 0, 0};
  int64_t nblend = 0;
  for (int64_t k = 0; k < m; ++k) {
    int64_t i = order[k];
    double dx = x - mean2d[2 * i];
    double dy = y - mean2d[2 * i + 1];
    double a = conic[3 * i], b = conic[3 * i + 1], c = conic[3 * i + 2];
    /* g = -1/2 d^T Q d and its screen derivatives */
    double g = -0.5 * (a * dx * dx + 2.0 * b * dx * dy + c * dy * dy);
    double gx = -(a * dx + b * dy);
    double gy = -(b * dx + c * dy);
    double gxy = -b;
    double alpha = opac[i] * exp(g);

    int skip = decide(alpha < cfg->alpha_min, fabs(alpha - cfg->alpha_min) / cfg->alpha_min,
                      cfg->tie_alpha, flip, nflip, k, OR_DEC_SKIP, amb, namb, amb_cap);
    if (skip) continue;
    int clamp = decide(alpha > cfg->alpha_max, fabs(alpha - cfg->alpha_max) / cfg->alpha_max,
                       cfg->tie_alpha, flip, nflip, k, OR_DEC_CLAMP, amb, namb, amb_cap);
    double ax, ay, axy;
    if (clamp) {
      alpha = cfg->alpha_max;
      ax = ay = axy = 0.0;
    } else {
      /* alpha = sigma e^g: d alpha/dx = alpha g_x, d2 alpha/dxdy = alpha (g_x g_y + g_xy) */
      ax = alpha * gx;
      ay = alpha * gy;
      axy = alpha * (gx * gy + gxy);
    }

    /* Front-to-back recurrences for B_i, A_i and their derivatives; T_i = 1 - A_{i-1}. */
    double T = 1.0 - A;
    for (int ch = 0; ch < 3; ++ch) {
      double ci = rgb[3 * i + ch];
      B[ch] = B[ch] + T * alpha * ci;
      Bx[ch] = Bx[ch] + ci * (T * ax - Ax * alpha);
      By[ch] = By[ch] + ci * (T * ay - Ay * alpha);
      Bxy[ch] = Bxy[ch] + ci * (T * axy - Ay * ax - Axy * alpha - Ax * ay);
    }
    double Axy_n = Axy * (1.0 - alpha) + T * axy - Ax * ay - Ay * ax;
    double Ax_n = Ax * (1.0 - alpha) + T * ax;
    double Ay_n = Ay * (1.0 - alpha) + T * ay;
    double A_n = A + alpha * T;
    A = A_n;
    Ax = Ax_n;
    Ay = Ay_n;
    Axy = Axy_n;
    ++nblend;

    double Tn = 1.0 - A;
    int stop = decide(Tn < cfg->t_min, fabs(Tn - cfg->t_min) / cfg->t_min, cfg->tie_t, flip,
                      nflip, k, OR_DEC_STOP, amb, namb, amb_cap);
    if (stop) break;
  }
  for (int ch = 0; ch < 3; ++ch) {
    out[ch] = B[ch] + (1.0 - A) * cfg->bg[ch];
    out[3 + ch] = Bx[ch] - Ax * cfg->bg[ch];
    out[6 + ch] = By[ch] - Ay * cfg->bg[ch];
    out[9 + ch] = Bxy[ch] - Axy * cfg->bg[ch];
  }
  return nblend;
}

/* Composite npts image points (px[p], py[p]) over the Gaussians order[0..m).
 *   out[p*12 ..]        I_rgb, I_x rgb, I_y rgb, I_xy rgb
 *   n_blend[p]          number of blended fragments
 *   n_amb[p]            number of near-tie decisions met on the reference walk
 * If variants != NULL, variants[p*8*12 ..] holds n_var[p] valid results:
 * the reference walk first, then every walk with a subset of the (at most
 * OR_MAX_AMB) near-tie decisions inverted.  n_var[p] = 0 marks a point with
 * more near ties than that (not checkable). */
void or_composite(int64_t m, const int64_t* order, const double* mean2d, const double* conic,
                  const double* opac, const double* rgb, const or_config* cfg, int64_t npts,
                  const double* px, const double* py, double* out, int64_t* n_blend,
                  int32_t* n_amb, double* variants, int32_t* n_var) {
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t p = 0; p < npts; ++p) {
    or_decision amb[OR_MAX_AMB];
    int namb = 0;
    double res[12];
    int64_t nb = walk(px[p], py[p], m, order, mean2d, conic, opac, rgb, cfg, NULL, 0, res, amb,
                      &namb, OR_MAX_AMB);
    memcpy(out + 12 * p, res, sizeof(res));
    if (n_blend) n_blend[p] = nb;
    if (n_amb) n_amb[p] = namb;
    if (variants) {
      double* v = variants + (int64_t)p * OR_MAX_VAR * 12;
      if (namb > OR_MAX_AMB) {
        n_var[p] = 0;
        continue;
      }
      memcpy(v, res, sizeof(res));
      int nv = 1;
      for (int mask = 1; mask < (1 << namb); ++mask) {
        or_decision fl[OR_MAX_AMB];
        int nf = 0;
        for (int b = 0; b < namb; ++b)
          if (mask & (1 << b)) fl[nf++] = amb[b];
        walk(px[p], py[p], m, order, mean2d, conic, opac, rgb, cfg, fl, nf, v + 12 * nv, NULL,
             NULL, 0);
        ++nv;
      }
      n_var[p] = nv;
    }
  }
}

/* ------------------------------------------------------------------------- */
/* Bicubic patches from values and derivatives                               */
/* ------------------------------------------------------------------------- */

/* The constant matrix C maps the coefficients (a0..a3) of a cubic to
 * (f(0), f(1), f'(0), f'(1)).  Its inverse is obtained by Gauss-Jordan
 * elimination with partial pivoting. */
static void build_C(double C[4][4]) {
  static const double Cv[4][4] = {{1, 0, 0, 0}, {1, 1, 1, 1}, {0, 1, 0, 0}, {0, 1, 2, 3}};
  memcpy(C, Cv, sizeof(Cv));
}

static void invert4(const double M[4][4], double Inv[4][4]) {
  double a[4][8];
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 8; ++c) a[r][c] = c < 4 ? M[r][c] : (c - 4 == r ? 1.0 : 0.0);
  for (int col = 0; col < 4; ++col) {
    int piv = col;
    for (int r = col + 1; r < 4; ++r)
      if (fabs(a[r][col]) > fabs(a[piv][col])) piv = r;
    if (piv != col)
      for (int c = 0; c < 8; ++c) {
        double tmp = a[col][c];
        a[col][c] = a[piv][c];
        a[piv][c] = tmp;
      }
    double d = a[col][col];
    for (int c = 0; c < 8; ++c) a[col][c] /= d;
    for (int r = 0; r < 4; ++r)
      if (r != col) {
        double f = a[r][col];
        for (int c = 0; c < 8; ++c) a[r][c] -= f * a[col][c];
      }
  }
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c) Inv[r][c] = a[r][c + 4];
}

void or_hermite_matrices(double* C_out, double* Cinv_out) {
  double C[4][4], Ci[4][4];
  build_C(C);
  invert4(C, Ci);
  memcpy(C_out, C, sizeof(C));
  memcpy(Cinv_out, Ci, sizeof(Ci));
}

/* Low-res buffer img is [h, w, 12] (I rgb, I_x rgb, I_y rgb, I_xy rgb).
 * At continuous low-res coordinates (u, v) the patch of cell (i, j),
 * i = clamp(floor(u), 0, w-2), j = clamp(floor(v), 0, h-2), is evaluated at
 * local (x, y) = (u - i, v - j) (outside [0,1] at the border: extrapolation).
 * out[p*12 ..] = p rgb, p_x rgb, p_y rgb, p_xy rgb (derivatives per low-res pixel). */
void or_patch_eval(const double* img, int32_t w, int32_t h, int64_t npts, const double* u,
                   const double* v, double* out) {
  double C[4][4], Ci[4][4];
  build_C(C);
  invert4(C, Ci);
#pragma omp parallel for schedule(static)
  for (int64_t p = 0; p < npts; ++p) {
    int i = (int)floor(u[p]);
    int j = (int)floor(v[p]);
    if (i < 0) i = 0;
    if (i > w - 2) i = w - 2;
    if (j < 0) j = 0;
    if (j > h - 2) j = h - 2;
    double x = u[p] - i, y = v[p] - j;
    double X[4] = {1, x, x * x, x * x * x}, Y[4] = {1, y, y * y, y * y * y};
    double dX[4] = {0, 1, 2 * x, 3 * x * x}, dY[4] = {0, 1, 2 * y, 3 * y * y};
    for (int ch = 0; ch < 3; ++ch) {
      /* corner (ox, oy) of the cell: value, f_x, f_y, f_xy */
#define PIX(ox, oy, q) img[(((int64_t)(j + (oy)) * w + (i + (ox))) * 12) + 3 * (q) + ch]
      double F[4][4] = {
          {PIX(0, 0, 0), PIX(0, 1, 0), PIX(0, 0, 2), PIX(0, 1, 2)},
          {PIX(1, 0, 0), PIX(1, 1, 0), PIX(1, 0, 2), PIX(1, 1, 2)},
          {PIX(0, 0, 1), PIX(0, 1, 1), PIX(0, 0, 3), PIX(0, 1, 3)},
          {PIX(1, 0, 1), PIX(1, 1, 1), PIX(1, 0, 3), PIX(1, 1, 3)},
      };
#undef PIX
      /* A = C^-1 F (C^T)^-1 */
      double CF[4][4], A[4][4];
      for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) {
          double acc = 0.0;
          for (int k = 0; k < 4; ++k) acc += Ci[r][k] * F[k][c];
          CF[r][c] = acc;
        }
      for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) {
          double acc = 0.0;
          for (int k = 0; k < 4; ++k) acc += CF[r][k] * Ci[c][k];
          A[r][c] = acc;
        }
      double pv = 0, px = 0, py = 0, pxy = 0;
      for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) {
          pv += X[r] * A[r][c] * Y[c];
          px += dX[r] * A[r][c] * Y[c];
          py += X[r] * A[r][c] * dY[c];
          pxy += dX[r] * A[r][c] * dY[c];
        }
      out[12 * p + ch] = pv;
      out[12 * p + 3 + ch] = px;
      out[12 * p + 6 + ch] = py;
      out[12 * p + 9 + ch] = pxy;
    }
  }
}

/* High-res pixel (X, Y) of a W x H target samples the low-res point
 * u = (X + 1/2) w / W - 1/2, v = (Y + 1/2) h / H - 1/2.  out[p*3 ..] = rgb. */
void or_upscale(const double* img, int32_t w, int32_t h, int32_t W, int32_t H, int64_t npts,
                const int32_t* X, const int32_t* Y, double* out) {
  const int64_t chunk = 4096;
  for (int64_t p0 = 0; p0 < npts; p0 += chunk) {
    int64_t cnt = npts - p0 < chunk ? npts - p0 : chunk;
    double* u = (double*)malloc(sizeof(double) * cnt);
    double* v = (double*)malloc(sizeof(double) * cnt);
    double* r = (double*)malloc(sizeof(double) * cnt * 12);
    for (int64_t k = 0; k < cnt; ++k) {
      u[k] = (X[p0 + k] + 0.5) * (double)w / (double)W - 0.5;
      v[k] = (Y[p0 + k] + 0.5) * (double)h / (double)H - 0.5;
    }
    or_patch_eval(img, w, h, cnt, u, v, r);
    for (int64_t k = 0; k < cnt; ++k)
      for (int ch = 0; ch < 3; ++ch) out[3 * (p0 + k) + ch] = r[12 * k + ch];
    free(u);
    free(v);
    free(r);
  }
}

/* ------------------------------------------------------------------------- */
/* Adjoints (gradients of a loss)                                            */
/* ------------------------------------------------------------------------- */

/* Gradient of L = sum_p g[p] . upscaled[p] (all W x H output pixels, rgb) with
 * respect to the low-res buffer [h, w, 12]: every output pixel evaluates
 * p = X^T C^-1 F C^-T Y, so the weight of F[k][c] is (C^-T X)_k (C^-T Y)_c;
 * it is added back to the image entry F[k][c] came from.  d_img is overwritten. */
void or_upscale_adjoint(const double* g, int32_t w, int32_t h, int32_t W, int32_t H,
                        double* d_img) {
  double C[4][4], Ci[4][4];
  build_C(C);
  invert4(C, Ci);
  memset(d_img, 0, sizeof(double) * (size_t)w * h * 12);
  for (int32_t Yp = 0; Yp < H; ++Yp)
    for (int32_t Xp = 0; Xp < W; ++Xp) {
      double u = (Xp + 0.5) * (double)w / (double)W - 0.5;
      double v = (Yp + 0.5) * (double)h / (double)H - 0.5;
      int i = (int)floor(u), j = (int)floor(v);
      if (i < 0) i = 0;
      if (i > w - 2) i = w - 2;
      if (j < 0) j = 0;
      if (j > h - 2) j = h - 2;
      double x = u - i, y = v - j;
      double X[4] = {1, x, x * x, x * x * x}, Y[4] = {1, y, y * y, y * y * y};
      double hx[4], hy[4];
      for (int k = 0; k < 4; ++k) {
        hx[k] = 0.0;
        hy[k] = 0.0;
        for (int r = 0; r < 4; ++r) {
          hx[k] += Ci[r][k] * X[r];
          hy[k] += Ci[r][k] * Y[r];
        }
      }
      /* F[k][c]: k = (x offset, value/x-derivative), c = (y offset, value/y-derivative),
       * laid out as in or_patch_eval: row k -> (ox, qx) = {(0,v),(1,v),(0,d),(1,d)} */
      static const int kox[4] = {0, 1, 0, 1}, kqd[4] = {0, 0, 1, 1};
      for (int k = 0; k < 4; ++k)
        for (int c = 0; c < 4; ++c) {
          int ox = kox[k], oy = kox[c];
          int q = kqd[k] + 2 * kqd[c];  /* 0 value, 1 f_x, 2 f_y, 3 f_xy */
          double wgt = hx[k] * hy[c];
          double* dst = d_img + (((int64_t)(j + oy) * w + (i + ox)) * 12) + 3 * q;
          const double* gp = g + 3 * ((int64_t)Yp * W + Xp);
          for (int ch = 0; ch < 3; ++ch) dst[ch] += wgt * gp[ch];
        }
    }
}

/* Gradient of L = sum_p G[p] . (I, I_x, I_y, I_xy)(px[p], py[p]) with respect
 * to the 2D parameters of every Gaussian, added to grad[i*9 ..] =
 * (mean x, mean y, conic a, b, c, opacity sigma, colour r, g, b).
 * The index set of each point (skips, clamps, stop) is that of the plain walk
 * and is held fixed; a clamped fragment (alpha = alpha_max) has no geometric
 * or opacity gradient.  The background enters as a last fragment of colour bg
 * and alpha 1, i.e. B-hat_{N+1} = bg. */
void or_composite_adjoint(int64_t m, const int64_t* order, const double* mean2d,
                          const double* conic, const double* opac, const double* rgb,
                          const or_config* cfg, int64_t npts, const double* px, const double* py,
                          const double* G, double* grad) {
  /* per blended fragment of one walk */
  int64_t* fi = (int64_t*)malloc(sizeof(int64_t) * (m > 0 ? m : 1));
  double* fs = (double*)malloc(sizeof(double) * 12 * (m > 0 ? m : 1));
  for (int64_t p = 0; p < npts; ++p) {
    const double x = px[p], y = py[p];
    const double* Gp = G + 12 * p;
    /* forward walk (front to back), recording alpha, its derivatives, and
     * A_{k-1} with its derivatives before each blend */
    double A = 0.0, Ax = 0.0, Ay = 0.0, Axy = 0.0;
    int64_t nf = 0;
    for (int64_t k = 0; k < m; ++k) {
      int64_t i = order[k];
      double dx = x - mean2d[2 * i], dy = y - mean2d[2 * i + 1];
      double a = conic[3 * i], b = conic[3 * i + 1], c = conic[3 * i + 2];
      double g = -0.5 * (a * dx * dx + 2.0 * b * dx * dy + c * dy * dy);
      double gx = -(a * dx + b * dy), gy = -(b * dx + c * dy), gxy = -b;
      double alpha = opac[i] * exp(g);
      if (alpha < cfg->alpha_min) continue;
      int clamp = alpha > cfg->alpha_max;
      double ax, ay, axy;
      if (clamp) {
        alpha = cfg->alpha_max;
        ax = ay = axy = 0.0;
      } else {
        ax = alpha * gx;
        ay = alpha * gy;
        axy = alpha * (gx * gy + gxy);
      }
      double* st = fs + 12 * nf;
      st[0] = alpha; st[1] = ax; st[2] = ay; st[3] = axy;
      st[4] = A; st[5] = Ax; st[6] = Ay; st[7] = Axy;
      st[8] = clamp; st[9] = dx; st[10] = dy; st[11] = 0.0;
      fi[nf++] = i;
      double T = 1.0 - A;
      double Axy_n = Axy * (1.0 - alpha) + T * axy - Ax * ay - Ay * ax;
      double Ax_n = Ax * (1.0 - alpha) + T * ax;
      double Ay_n = Ay * (1.0 - alpha) + T * ay;
      A = A + alpha * T;
      Ax = Ax_n;
      Ay = Ay_n;
      Axy = Axy_n;
      if (1.0 - A < cfg->t_min) break;
    }
    /* backward walk (back to front): B-hat_{k+1} and its derivatives */
    double Bh[3], Bhx[3] = {0, 0, 0}, Bhy[3] = {0, 0, 0}, Bhxy[3] = {0, 0, 0};
    for (int ch = 0; ch < 3; ++ch) Bh[ch] = cfg->bg[ch];
    for (int64_t f = nf - 1; f >= 0; --f) {
      const int64_t i = fi[f];
      const double* st = fs + 12 * f;
      const double alpha = st[0], ax = st[1], ay = st[2], axy = st[3];
      const double Ak = st[4], Akx = st[5], Aky = st[6], Akxy = st[7];
      const int clamp = st[8] != 0.0;
      const double dx = st[9], dy = st[10];
      const double T = 1.0 - Ak;
      /* colour: weights of c_k in I, I_x, I_y, I_xy */
      const double w0 = T * alpha, wx = T * ax - Akx * alpha, wy = T * ay - Aky * alpha;
      const double wxy = T * axy - Akx * ay - Aky * ax - Akxy * alpha;
      for (int ch = 0; ch < 3; ++ch)
        grad[9 * i + 6 + ch] += Gp[ch] * w0 + Gp[3 + ch] * wx + Gp[6 + ch] * wy + Gp[9 + ch] * wxy;
      if (!clamp) {
        /* dI/d alpha_k = T_k (c_k - B-hat_{k+1}) and its screen derivatives */
        double P[3], Px[3], Py[3], Pxy[3];
        for (int ch = 0; ch < 3; ++ch) {
          const double e = rgb[3 * i + ch] - Bh[ch];
          P[ch] = T * e;
          Px[ch] = -Akx * e - T * Bhx[ch];
          Py[ch] = -Aky * e - T * Bhy[ch];
          Pxy[ch] = -Akxy * e - T * Bhxy[ch] + Akx * Bhy[ch] + Aky * Bhx[ch];
        }
        /* alpha = sigma e^g and the derivatives of alpha, alpha_x, alpha_y,
         * alpha_xy with respect to (mean x, mean y, a, b, c, sigma) */
        const double a = conic[3 * i], b = conic[3 * i + 1], c = conic[3 * i + 2];
        const double gx = -(a * dx + b * dy), gy = -(b * dx + c * dy), gxy = -b;
        /* g_theta, gx_theta, gy_theta, gxy_theta */
        const double dg[5][4] = {
            {a * dx + b * dy, a, b, 0.0},        /* mean x: d(dx) = -1 */
            {b * dx + c * dy, b, c, 0.0},        /* mean y */
            {-0.5 * dx * dx, -dx, 0.0, 0.0},     /* a */
            {-dx * dy, -dy, -dx, -1.0},          /* b */
            {-0.5 * dy * dy, 0.0, -dy, 0.0},     /* c */
        };
        for (int t = 0; t < 6; ++t) {
          double at, axt, ayt, axyt;
          if (t < 5) {
            at = alpha * dg[t][0];
            axt = at * gx + alpha * dg[t][1];
            ayt = at * gy + alpha * dg[t][2];
            axyt = at * (gx * gy + gxy) + alpha * (dg[t][1] * gy + gx * dg[t][2] + dg[t][3]);
          } else {
            const double sg = opac[i];
            at = alpha / sg;
            axt = ax / sg;
            ayt = ay / sg;
            axyt = axy / sg;
          }
          double acc = 0.0;
          for (int ch = 0; ch < 3; ++ch) {
            acc += Gp[ch] * (P[ch] * at);
            acc += Gp[3 + ch] * (Px[ch] * at + P[ch] * axt);
            acc += Gp[6 + ch] * (Py[ch] * at + P[ch] * ayt);
            acc += Gp[9 + ch] * (Pxy[ch] * at + Px[ch] * ayt + Py[ch] * axt + P[ch] * axyt);
          }
          grad[9 * i + t] += acc;
        }
      }
      /* B-hat_k from B-hat_{k+1} */
      for (int ch = 0; ch < 3; ++ch) {
        const double ci = rgb[3 * i + ch];
        const double e = ci - Bh[ch];
        const double nBxy = (1.0 - alpha) * Bhxy[ch] + axy * e - ay * Bhx[ch] - ax * Bhy[ch];
        const double nBx = (1.0 - alpha) * Bhx[ch] + ax * e;
        const double nBy = (1.0 - alpha) * Bhy[ch] + ay * e;
        Bh[ch] = (1.0 - alpha) * Bh[ch] + alpha * ci;
        Bhx[ch] = nBx;
        Bhy[ch] = nBy;
        Bhxy[ch] = nBxy;
      }
    }
  }
  free(fi);
  free(fs);
}

int32_t or_max_variants(void) { return OR_MAX_VAR; }

#ifdef _OPENMP
#include <omp.h>
#endif
/* Threads an OpenMP region of the oracle uses. */
int32_t or_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
