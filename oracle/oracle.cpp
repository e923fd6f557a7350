// FP64 reference ("oracle") of the differentiable Gaussian-splatting tile rasterizer.
//
// TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
// leg of the benchmark load this library.  It shares no code with the HIP path.
//
// What it computes (paper: Trick-GS, arXiv 2501.14534):
//   * projection of 3D Gaussians to 2D screen-space Gaussians with the EWA
//     Jacobian (Sec. 3.1, Eq. 1) and the low-pass dilation Sigma' + sI
//     (Sec. 3.2.4, "progressive training by scales");
//   * the learned per-Gaussian volume mask applied to opacity and scales
//     (Sec. 3.2.1, Eq. 3) and the per-band SH mask (Sec. 3.2.3, Eq. 5), both
//     hard-thresholded in the forward pass with straight-through gradients;
//   * view-dependent colour from the diffuse colour plus SH bands 1..3, kept
//     as separate inputs (Sec. 3.2.5);
//   * front-to-back alpha compositing of depth-ordered Gaussians (Eq. 2);
//   * the gradient of the composited image with respect to every raw input.
// Where the paper is silent (pinhole conventions, the compositing constants,
// the tile/binning rule, ordering ties) the oracle follows the readings listed
// in the design notes; each is named at the point of use below.
//
// Plain by construction: per-pixel walks in list order, std::sort for the
// (tile, depth, id) order, and forward-mode dual numbers for the derivative of
// the projection and colour, so the backward of those stages is the exact
// derivative of the very code that computes their forward values.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

extern "C" {

struct OrcGaussians {
  const double* means;           // [3][n]
  const double* log_scales;      // [3][n]
  const double* quats;           // [4][n] w, x, y, z (need not be normalised)
  const double* opacity_logits;  // [n]
  const double* sh_dc;           // [3][n] diffuse colour (band 0)
  const double* sh_rest;         // [(K-1)][3][n], K = (deg+1)^2; NULL when deg == 0
  const double* mask_logits;     // [n] or NULL
  const double* sh_mask_logits;  // [3][n] (bands 1..3) or NULL
  int64_t n;
  int32_t sh_degree;
  int32_t pad_;
  double mask_eps;
  double sh_mask_eps;
};

struct OrcCamera {
  double R[9];  // world -> camera, row-major; camera x right, y down, z forward
  double t[3];
  double fx, fy, cx, cy;
  int32_t width, height;
};

struct OrcOpts {
  double near_plane;
  double tan_clamp;
  double lowpass;
  double bg[3];
  int32_t tile_w, tile_h;
  int32_t lowpass_progressive;
};

struct OrcGrads {  // accumulated (+=); NULL members are skipped
  double* means;
  double* log_scales;
  double* quats;
  double* opacity_logits;
  double* sh_dc;
  double* sh_rest;
  double* mask_logits;
  double* sh_mask_logits;
};

}  // extern "C"

namespace {

// ---------------------------------------------------------------------------
// Compositing constants (not in the paper; the 3DGS rasterizer it builds on):
// alpha cap 0.99, skip below 1/255, stop once transmittance would fall under
// 1e-4.  The rule is defined with the single-precision values of the three
// constants, which the oracle uses exactly.
const double kAlphaMax = (double)0.99f;
const double kAlphaMin = (double)(1.0f / 255.0f);
const double kTMin = (double)1e-4f;

// ---------------------------------------------------------------------------
// Forward-mode dual numbers: value + gradient with respect to NV inputs.
template <int NV>
struct Dual {
  double v;
  double d[NV];
  Dual() : v(0.0) { std::memset(d, 0, sizeof(d)); }
  Dual(double x) : v(x) { std::memset(d, 0, sizeof(d)); }  // NOLINT: implicit on purpose
  static Dual var(double x, int i) {
    Dual r(x);
    r.d[i] = 1.0;
    return r;
  }
};

template <int NV> Dual<NV> operator+(const Dual<NV>& a, const Dual<NV>& b) {
  Dual<NV> r; r.v = a.v + b.v;
  for (int i = 0; i < NV; ++i) r.d[i] = a.d[i] + b.d[i];
  return r;
}
template <int NV> Dual<NV> operator-(const Dual<NV>& a, const Dual<NV>& b) {
  Dual<NV> r; r.v = a.v - b.v;
  for (int i = 0; i < NV; ++i) r.d[i] = a.d[i] - b.d[i];
  return r;
}
template <int NV> Dual<NV> operator-(const Dual<NV>& a) {
  Dual<NV> r; r.v = -a.v;
  for (int i = 0; i < NV; ++i) r.d[i] = -a.d[i];
  return r;
}
template <int NV> Dual<NV> operator*(const Dual<NV>& a, const Dual<NV>& b) {
  Dual<NV> r; r.v = a.v * b.v;
  for (int i = 0; i < NV; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
  return r;
}
template <int NV> Dual<NV> operator/(const Dual<NV>& a, const Dual<NV>& b) {
  Dual<NV> r; r.v = a.v / b.v;
  for (int i = 0; i < NV; ++i) r.d[i] = (a.d[i] * b.v - a.v * b.d[i]) / (b.v * b.v);
  return r;
}
template <int NV> Dual<NV> operator+(const Dual<NV>& a, double b) { return a + Dual<NV>(b); }
template <int NV> Dual<NV> operator+(double a, const Dual<NV>& b) { return Dual<NV>(a) + b; }
template <int NV> Dual<NV> operator-(const Dual<NV>& a, double b) { return a - Dual<NV>(b); }
template <int NV> Dual<NV> operator-(double a, const Dual<NV>& b) { return Dual<NV>(a) - b; }
template <int NV> Dual<NV> operator*(const Dual<NV>& a, double b) { return a * Dual<NV>(b); }
template <int NV> Dual<NV> operator*(double a, const Dual<NV>& b) { return Dual<NV>(a) * b; }
template <int NV> Dual<NV> operator/(const Dual<NV>& a, double b) { return a / Dual<NV>(b); }
template <int NV> Dual<NV> operator/(double a, const Dual<NV>& b) { return Dual<NV>(a) / b; }
template <int NV> Dual<NV> exp(const Dual<NV>& a) {
  Dual<NV> r; r.v = std::exp(a.v);
  for (int i = 0; i < NV; ++i) r.d[i] = r.v * a.d[i];
  return r;
}
template <int NV> Dual<NV> sqrt(const Dual<NV>& a) {
  Dual<NV> r; r.v = std::sqrt(a.v);
  for (int i = 0; i < NV; ++i) r.d[i] = a.d[i] / (2.0 * r.v);
  return r;
}

inline double val(double x) { return x; }
template <int NV> inline double val(const Dual<NV>& x) { return x.v; }
inline double exp(double x) { return std::exp(x); }
inline double sqrt(double x) { return std::sqrt(x); }

// Clamp of x to [lo, hi]: a clamped value carries no derivative.
template <class S> S clampd(const S& x, double lo, double hi) {
  if (val(x) < lo) return S(lo);
  if (val(x) > hi) return S(hi);
  return x;
}

template <class S> S sigmoid(const S& x) { return 1.0 / (1.0 + exp(-x)); }

// Straight-through estimator of Eq. 3 / Eq. 5:
//   M = sg(1(sigma(m) > eps) - sigma(m)) + sigma(m)
// Forward value is the hard indicator; the derivative is that of sigma(m).
inline double ste(double hard, double /*soft*/) { return hard; }
template <int NV> Dual<NV> ste(double hard, const Dual<NV>& soft) {
  Dual<NV> r = soft;
  r.v = hard;
  return r;
}

// ---------------------------------------------------------------------------
// Real spherical harmonics, degree <= 3, Condon-Shortley phase kept in the
// real basis (Y_{l,m>0} = sqrt2 Re Y_l^m, Y_{l,m<0} = sqrt2 Im Y_l^|m|).
// Coefficient index k = l*l + l + m.  Constants are the closed forms.
template <class S>
void sh_basis(const S& x, const S& y, const S& z, S Y[16]) {
  const double pi = M_PI;
  const double c0 = 0.5 * std::sqrt(1.0 / pi);
  const double c1 = std::sqrt(3.0 / (4.0 * pi));
  const double c2a = 0.5 * std::sqrt(15.0 / pi);
  const double c2b = 0.25 * std::sqrt(5.0 / pi);
  const double c2c = 0.25 * std::sqrt(15.0 / pi);
  const double c3a = 0.25 * std::sqrt(35.0 / (2.0 * pi));
  const double c3b = 0.5 * std::sqrt(105.0 / pi);
  const double c3c = 0.25 * std::sqrt(21.0 / (2.0 * pi));
  const double c3d = 0.25 * std::sqrt(7.0 / pi);
  const double c3e = 0.25 * std::sqrt(105.0 / pi);
  S xx = x * x, yy = y * y, zz = z * z;
  Y[0] = S(c0);
  Y[1] = -c1 * y;
  Y[2] = c1 * z;
  Y[3] = -c1 * x;
  Y[4] = c2a * (x * y);
  Y[5] = -c2a * (y * z);
  Y[6] = c2b * (2.0 * zz - xx - yy);
  Y[7] = -c2a * (x * z);
  Y[8] = c2c * (xx - yy);
  Y[9] = -c3a * (y * (3.0 * xx - yy));
  Y[10] = c3b * (x * y * z);
  Y[11] = -c3c * (y * (4.0 * zz - xx - yy));
  Y[12] = c3d * (z * (2.0 * zz - 3.0 * xx - 3.0 * yy));
  Y[13] = -c3c * (x * (4.0 * zz - xx - yy));
  Y[14] = c3e * (z * (xx - yy));
  Y[15] = -c3a * (x * (xx - 3.0 * yy));
}

// ---------------------------------------------------------------------------
// Geometry of one Gaussian in one view.
//   inputs : mean mu, log-scales, quaternion q (w,x,y,z), opacity logit, mask logit
//   outputs: screen mean (u, v), conic (A, B, C) = inverse of Sigma' (so the
//            exponent of Eq. 1 is -(A dx^2 + 2B dx dy + C dy^2)/2), masked
//            opacity o', camera depth, Sigma' itself and the integer radius.
// Returns false when the Gaussian is culled.
template <class S>
struct Geom {
  S u, v, A, B, C, op;
  S cov[3];  // Sigma' + sI: a, b, c
  double depth;
  int radius;
};

template <class S>
bool project_geom(const S mu[3], const S logs[3], const S q[4], const S& op_logit, const S* mask_logit,
                  double mask_eps, const OrcCamera& cam, const OrcOpts& o, Geom<S>* out) {
  // Volume mask (Eq. 3) on opacity and scales (Sec. 3.2.1).  A Gaussian whose
  // hard mask is 0 contributes nothing, so it is culled here.
  S M(1.0);
  if (mask_logit) {
    S soft = sigmoid(*mask_logit);
    double hard = val(soft) > mask_eps ? 1.0 : 0.0;
    if (hard == 0.0) return false;
    M = ste(hard, soft);
  }
  // World -> camera; depth is the camera-space z of the mean; near-plane cull.
  const double* R = cam.R;
  S t[3];
  for (int i = 0; i < 3; ++i) t[i] = R[3 * i] * mu[0] + R[3 * i + 1] * mu[1] + R[3 * i + 2] * mu[2] + cam.t[i];
  if (!(val(t[2]) > o.near_plane)) return false;

  // 3D covariance Sigma = Rq diag(s'^2) Rq^T from the normalised quaternion.
  S s[3];
  for (int k = 0; k < 3; ++k) s[k] = M * exp(logs[k]);
  S qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  if (!(val(qn) > 0.0) || !std::isfinite(val(qn))) return false;
  S w = q[0] / qn, x = q[1] / qn, y = q[2] / qn, z = q[3] / qn;
  S Rq[3][3] = {
      {1.0 - 2.0 * (y * y + z * z), 2.0 * (x * y - w * z), 2.0 * (x * z + w * y)},
      {2.0 * (x * y + w * z), 1.0 - 2.0 * (x * x + z * z), 2.0 * (y * z - w * x)},
      {2.0 * (x * z - w * y), 2.0 * (y * z + w * x), 1.0 - 2.0 * (x * x + y * y)}};
  S Sig[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      S acc(0.0);
      for (int k = 0; k < 3; ++k) acc = acc + Rq[i][k] * Rq[j][k] * (s[k] * s[k]);
      Sig[i][j] = acc;
    }

  // EWA (Eq. 1): Jacobian of the perspective map at the mean.  The lateral
  // ratios are clamped to tan_clamp times the half field of view (a guard for
  // Gaussians far off screen; clamped ratios carry no derivative).
  const double limx = o.tan_clamp * 0.5 * cam.width / cam.fx;
  const double limy = o.tan_clamp * 0.5 * cam.height / cam.fy;
  S rx = clampd(t[0] / t[2], -limx, limx);
  S ry = clampd(t[1] / t[2], -limy, limy);
  S J[2][3] = {{cam.fx / t[2], S(0.0), -cam.fx * rx / t[2]}, {S(0.0), cam.fy / t[2], -cam.fy * ry / t[2]}};
  S Tm[2][3];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 3; ++j) Tm[i][j] = J[i][0] * R[j] + J[i][1] * R[3 + j] + J[i][2] * R[6 + j];
  S c2[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      S acc(0.0);
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) acc = acc + Tm[i][a] * Sig[a][b] * Tm[j][b];
      c2[i][j] = acc;
    }
  // Low-pass dilation Sigma' + sI (added to both diagonal entries).
  S a = c2[0][0] + o.lowpass, b = c2[0][1], c = c2[1][1] + o.lowpass;
  S det = a * c - b * b;
  if (!(val(det) > 0.0)) return false;
  out->A = c / det;
  out->B = -b / det;
  out->C = a / det;
  out->cov[0] = a;
  out->cov[1] = b;
  out->cov[2] = c;
  // Screen-space extent: 3 standard deviations along the major axis.
  double mid = 0.5 * (val(a) + val(c));
  double lam = mid + std::sqrt(std::max(0.0, mid * mid - val(det)));
  out->radius = (int)std::ceil(3.0 * std::sqrt(lam));
  out->u = cam.fx * t[0] / t[2] + cam.cx;
  out->v = cam.fy * t[1] / t[2] + cam.cy;
  out->op = M * sigmoid(op_logit);
  out->depth = val(t[2]);
  return true;
}

// View-dependent colour: diffuse colour plus SH bands 1..deg, each band scaled
// by its hard mask (Eq. 5: c^l <- M^l c^l), clamped below at 0.
template <class S>
void colour(const S mu[3], const S dc[3], const S (*rest)[3], const S* bmask, double sh_eps, int deg,
            const double campos[3], S rgb[3]) {
  S d[3] = {mu[0] - campos[0], mu[1] - campos[1], mu[2] - campos[2]};
  S len = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  S Y[16];
  sh_basis(d[0] / len, d[1] / len, d[2] / len, Y);
  S band_m[4] = {S(1.0), S(1.0), S(1.0), S(1.0)};
  if (bmask)
    for (int l = 1; l <= 3; ++l) {
      S soft = sigmoid(bmask[l - 1]);
      band_m[l] = ste(val(soft) > sh_eps ? 1.0 : 0.0, soft);
    }
  for (int ch = 0; ch < 3; ++ch) {
    S acc = dc[ch];
    for (int l = 1; l <= deg; ++l) {
      S band(0.0);
      for (int k = l * l; k < (l + 1) * (l + 1); ++k) band = band + Y[k] * rest[k - 1][ch];
      acc = acc + band_m[l] * band;
    }
    rgb[ch] = val(acc) < 0.0 ? S(0.0) : acc;
  }
}

inline void campos_of(const OrcCamera& cam, double p[3]) {
  // camera centre = -R^T t
  for (int j = 0; j < 3; ++j) p[j] = -(cam.R[j] * cam.t[0] + cam.R[3 + j] * cam.t[1] + cam.R[6 + j] * cam.t[2]);
}

// A Gaussian is culled when any input that its forward value reads is not finite.
bool finite_inputs(const OrcGaussians& g, int64_t i) {
  const int64_t n = g.n;
  for (int k = 0; k < 3; ++k)
    if (!std::isfinite(g.means[k * n + i]) || !std::isfinite(g.log_scales[k * n + i]) ||
        !std::isfinite(g.sh_dc[k * n + i]))
      return false;
  for (int k = 0; k < 4; ++k)
    if (!std::isfinite(g.quats[k * n + i])) return false;
  if (!std::isfinite(g.opacity_logits[i])) return false;
  if (g.mask_logits && !std::isfinite(g.mask_logits[i])) return false;
  // SH band l's coefficients enter the forward only when its hard mask is on
  bool on[4] = {true, true, true, true};
  if (g.sh_mask_logits && g.sh_degree > 0)
    for (int l = 1; l <= 3; ++l) {
      const double m = g.sh_mask_logits[(l - 1) * n + i];
      if (!std::isfinite(m)) return false;
      on[l] = 1.0 / (1.0 + std::exp(-m)) > g.sh_mask_eps;
    }
  for (int l = 1; l <= g.sh_degree; ++l) {
    if (!on[l]) continue;
    for (int k = l * l; k < (l + 1) * (l + 1); ++k)
      for (int c = 0; c < 3; ++c)
        if (!std::isfinite(g.sh_rest[((k - 1) * 3 + c) * n + i])) return false;
  }
  return true;
}

struct ViewGeom {
  int W, H, TX, TY;
  int64_t tile_off, pix_off;
};

std::vector<ViewGeom> view_table(int V, const OrcCamera* cams, const OrcOpts& o, int64_t* total_tiles,
                                 int64_t* total_pix) {
  std::vector<ViewGeom> vt(V);
  int64_t to = 0, po = 0;
  for (int v = 0; v < V; ++v) {
    ViewGeom& g = vt[v];
    g.W = cams[v].width;
    g.H = cams[v].height;
    g.TX = (g.W + o.tile_w - 1) / o.tile_w;
    g.TY = (g.H + o.tile_h - 1) / o.tile_h;
    g.tile_off = to;
    g.pix_off = po;
    to += (int64_t)g.TX * g.TY;
    po += (int64_t)g.W * g.H;
  }
  if (total_tiles) *total_tiles = to;
  if (total_pix) *total_pix = po;
  return vt;
}

struct Contrib {  // one composited (pixel, entry) pair
  int64_t entry;
  uint32_t rec;
  double alpha, T, G, dx, dy;
  bool clamped;
};

// The per-pixel walk of Eq. 2 over the tile's ordered list.  Fills `list`
// with the composited pairs; returns the final transmittance.
struct WalkResult {
  double C[3];
  double T;
  int32_t last;
  uint8_t flags;
  uint64_t hash;
};

// Near-threshold flags (the decision-consistency protocol; not part of the
// function itself).  eps[0..5]: a decision is flagged when the compared
// quantity lies within its window of the threshold, the window being the
// rounding a single-precision evaluation of the same quantity can carry:
//   alpha (skip, cap):  relative  eps[0] + eps[3] S, where S = |A| dx^2/2 +
//                       |B dx dy| + |C| dy^2/2 bounds the exponent's terms;
//   T (1 - alpha) (stop): relative eps[1] + e_T + the (1 - alpha) part, e_T
//                       accumulating eps[4] + w_alpha alpha / (1 - alpha) per
//                       composited Gaussian;
//   square edge:        eps[2] + eps[5] |dx| pixels, but never when px - u
//                       is exact in single precision (the test is then exact);
//   radius (rec_flags bit 1, a record whose 3 sqrt(lambda) is near an
//                       integer): the pixel is within one pixel of its square.
// When the records themselves carry rounding (an independent run compared
// with another precision's projection), rec_win[2 rec] is the record's
// screen-position error in pixels, widening the square-edge window and the
// alpha window by its effect on the exponent, and rec_win[2 rec + 1] its
// conic's relative error, widening the alpha window by that fraction of S;
// depth[rec] (with eps[6], a relative window) flags two consecutive records
// that reach the pixel at depths within the window (their order may differ).
// Flag bits per pixel: 1 square edge, 2 alpha skip, 4 termination, 8 alpha
// cap, 16 near-integer radius, 32 near-equal depths.
bool f32_exact(double x) { return (double)(float)x == x; }

struct FlagInputs {
  const double* eps;       // [7] or NULL: no flags
  const uint8_t* rec;      // per record, bit 1: radius near an integer; or NULL
  const double* rec_win;   // per record (position px, conic relative), or NULL
  const double* depth;     // per record, or NULL
};

WalkResult walk_pixel(double px, double py, int64_t start, int64_t end, const uint32_t* ids, const double* uv,
                      const double* conic, const double* opacity, const double* rgb, const int32_t* radius,
                      const FlagInputs& fi, std::vector<Contrib>* list) {
  const double* eps = fi.eps;
  const uint8_t* rec_flags = fi.rec;
  WalkResult r;
  r.C[0] = r.C[1] = r.C[2] = 0.0;
  r.T = 1.0;
  r.last = 0;
  r.flags = 0;
  r.hash = 1469598103934665603ull;
  double eT = eps ? eps[1] : 0.0;  // relative window of the transmittance reached so far
  double prev_depth = -1.0;        // depth of the last record that reached the pixel
  for (int64_t j = start; j < end; ++j) {
    const uint32_t rec = ids[j];
    const double dx = px - uv[2 * rec], dy = py - uv[2 * rec + 1];
    const double rad = (double)radius[rec];
    const double A = conic[3 * rec], B = conic[3 * rec + 1], Cc = conic[3 * rec + 2];
    const double q = A * dx * dx + 2.0 * B * dx * dy + Cc * dy * dy;
    const double G = std::exp(-0.5 * q);
    const double raw = opacity[rec] * G;
    const double alpha = std::min(kAlphaMax, raw);
    const bool inside = std::fabs(dx) <= rad && std::fabs(dy) <= rad;
    double wa = 0.0, wq = 0.0;  // relative windows of alpha and of (1 - alpha)
    if (eps) {
      const double S = 0.5 * std::fabs(A) * dx * dx + std::fabs(B * dx * dy) + 0.5 * std::fabs(Cc) * dy * dy;
      const double ep = fi.rec_win ? fi.rec_win[2 * rec] : 0.0;
      const double ec = fi.rec_win ? fi.rec_win[2 * rec + 1] : 0.0;
      const double dq = ep * (std::fabs(A * dx + B * dy) + std::fabs(B * dx + Cc * dy)) + 0.5 * ep * ep * (std::fabs(A) + 2.0 * std::fabs(B) + std::fabs(Cc));
      wa = eps[0] + eps[3] * S + ec * S + dq;
      wa = wa < 0.5 ? wa : 0.5;
      wq = alpha < 1.0 ? wa * alpha / (1.0 - alpha) : 0.0;
      const bool reach = alpha >= kAlphaMin * (1.0 - wa);
      const double edx = eps[2] + eps[5] * std::fabs(dx) + ep, edy = eps[2] + eps[5] * std::fabs(dy) + ep;
      const bool ex = std::fabs(std::fabs(dx) - rad) <= edx && (ep > 0.0 || !f32_exact(dx));
      const bool ey = std::fabs(std::fabs(dy) - rad) <= edy && (ep > 0.0 || !f32_exact(dy));
      if ((ex || ey) && reach) r.flags |= 1;
      if (rec_flags && (rec_flags[rec] & 1) && reach && std::fabs(dx) <= rad + 1.0 && std::fabs(dy) <= rad + 1.0 &&
          (std::fabs(dx) >= rad - 1.0 || std::fabs(dy) >= rad - 1.0))
        r.flags |= 16;
      if (fi.depth && reach && std::fabs(dx) <= rad + ep + 1e-6 && std::fabs(dy) <= rad + ep + 1e-6) {
        const double d = fi.depth[rec];
        if (prev_depth >= 0.0 && std::fabs(d - prev_depth) <= eps[6] * d) r.flags |= 32;
        prev_depth = d;
      }
    }
    // Square test: the pixel centre must lie in the Gaussian's closed screen
    // square of half-side `radius` (keeps the result independent of tiling).
    if (!inside) continue;
    if (eps && std::fabs(alpha - kAlphaMin) <= wa * kAlphaMin) r.flags |= 2;
    if (alpha < kAlphaMin) continue;
    const double Tn = r.T * (1.0 - alpha);
    if (eps && std::fabs(Tn - kTMin) <= (eT + wq + eps[4]) * kTMin) r.flags |= 4;
    if (eps && std::fabs(raw - kAlphaMax) <= wa * kAlphaMax) r.flags |= 8;
    if (eps) eT += wq + eps[4];
    if (Tn < kTMin) {  // stop before compositing this Gaussian
      r.hash = (r.hash ^ (uint64_t)(j - start + 1) * 0x9E3779B97F4A7C15ull) * 1099511628211ull;
      break;
    }
    if (list) list->push_back(Contrib{j, rec, alpha, r.T, G, dx, dy, raw > kAlphaMax});
    for (int ch = 0; ch < 3; ++ch) r.C[ch] += rgb[3 * rec + ch] * alpha * r.T;
    r.T = Tn;
    r.last = (int32_t)(j - start + 1);
    r.hash = (r.hash ^ ((uint64_t)(j - start) * 2 + (raw > kAlphaMax ? 1 : 0))) * 1099511628211ull;
  }
  return r;
}

}  // namespace

extern "C" {

int orc_num_threads() {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void orc_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

// Real SH basis (16 functions) at m unit directions [m][3] -> out [m][16].
void orc_sh_basis(int64_t m, const double* dirs, double* out) {
  for (int64_t i = 0; i < m; ++i) sh_basis(dirs[3 * i], dirs[3 * i + 1], dirs[3 * i + 2], out + 16 * i);
}

// 3D covariance (upper triangle xx, xy, xz, yy, yz, zz) of each Gaussian, masks ignored.
void orc_cov3d(const OrcGaussians* g, double* out) {
  const int64_t n = g->n;
  for (int64_t i = 0; i < n; ++i) {
    double q[4], s[3];
    for (int k = 0; k < 4; ++k) q[k] = g->quats[k * n + i];
    for (int k = 0; k < 3; ++k) s[k] = std::exp(g->log_scales[k * n + i]);
    double qn = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    double w = q[0] / qn, x = q[1] / qn, y = q[2] / qn, z = q[3] / qn;
    double Rq[3][3] = {{1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)},
                       {2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)},
                       {2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)}};
    int o = 0;
    for (int a = 0; a < 3; ++a)
      for (int b = a; b < 3; ++b) {
        double acc = 0;
        for (int k = 0; k < 3; ++k) acc += Rq[a][k] * Rq[b][k] * s[k] * s[k];
        out[6 * i + o++] = acc;
      }
  }
}

// Projection of all n Gaussians into one view.
//   valid [n]; uv [n][2]; conic [n][3]; depth [n]; radius [n]; opacity [n]
//   (masked o'); rgb [n][3]; cov2d [n][3] (Sigma' + sI; may be NULL).
// Options of one view.  With progressive scaling (Sec. 3.2.4) the low-pass s
// of the view is HW / (9 pi N) for N Gaussians -- each projected Gaussian then
// covers at least 9 pi s, the share of the image that N Gaussians fill --
// bounded below by the given s (0.3).
OrcOpts view_opts(const OrcOpts& o, const OrcCamera& c, int64_t n) {
  OrcOpts e = o;
  if (o.lowpass_progressive && n > 0)
    e.lowpass = std::max(o.lowpass, (double)c.width * (double)c.height / (9.0 * M_PI * (double)n));
  return e;
}

// Culled Gaussians get valid = 0 and zeros elsewhere.
void orc_project(const OrcGaussians* g, const OrcCamera* cam, const OrcOpts* o, int32_t* valid, double* uv,
                 double* conic, double* depth, int32_t* radius, double* opacity, double* rgb, double* cov2d) {
  const int64_t n = g->n;
  double campos[3];
  campos_of(*cam, campos);
  const int deg = g->sh_degree;
  const OrcOpts ov = view_opts(*o, *cam, n);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    valid[i] = 0;
    uv[2 * i] = uv[2 * i + 1] = 0;
    conic[3 * i] = conic[3 * i + 1] = conic[3 * i + 2] = 0;
    depth[i] = 0;
    radius[i] = 0;
    opacity[i] = 0;
    rgb[3 * i] = rgb[3 * i + 1] = rgb[3 * i + 2] = 0;
    if (cov2d) cov2d[3 * i] = cov2d[3 * i + 1] = cov2d[3 * i + 2] = 0;
    if (!finite_inputs(*g, i)) continue;
    double mu[3], ls[3], q[4], ml;
    for (int k = 0; k < 3; ++k) mu[k] = g->means[k * n + i], ls[k] = g->log_scales[k * n + i];
    for (int k = 0; k < 4; ++k) q[k] = g->quats[k * n + i];
    if (g->mask_logits) ml = g->mask_logits[i];
    Geom<double> ge;
    if (!project_geom<double>(mu, ls, q, g->opacity_logits[i], g->mask_logits ? &ml : nullptr, g->mask_eps, *cam,
                              ov, &ge))
      continue;
    double dc[3], rest[15][3], bm[3], col[3];
    for (int c = 0; c < 3; ++c) dc[c] = g->sh_dc[c * n + i];
    const int K = (deg + 1) * (deg + 1);
    for (int k = 1; k < K; ++k)
      for (int c = 0; c < 3; ++c) rest[k - 1][c] = g->sh_rest[((k - 1) * 3 + c) * n + i];
    if (g->sh_mask_logits)
      for (int l = 0; l < 3; ++l) bm[l] = g->sh_mask_logits[l * n + i];
    colour<double>(mu, dc, rest, g->sh_mask_logits ? bm : nullptr, g->sh_mask_eps, deg, campos, col);
    valid[i] = 1;
    uv[2 * i] = ge.u;
    uv[2 * i + 1] = ge.v;
    conic[3 * i] = ge.A;
    conic[3 * i + 1] = ge.B;
    conic[3 * i + 2] = ge.C;
    depth[i] = ge.depth;
    radius[i] = ge.radius;
    opacity[i] = ge.op;
    for (int c = 0; c < 3; ++c) rgb[3 * i + c] = col[c];
    if (cov2d)
      for (int c = 0; c < 3; ++c) cov2d[3 * i + c] = val(ge.cov[c]);
  }
}

// Tile binning and (tile, depth, id) ordering for V views of n Gaussians.
// Inputs are per record r = view * n + gaussian, in single precision, as the
// rule is defined on single-precision screen positions:
//   tile rect x: [floor((u - r)/TW), floor((u + r)/TW)] clipped to the grid,
//   where u - r and u + r are single IEEE float operations and TW is a power
//   of two (exact scaling); likewise y.  Area 0 means not binned.
// Key of a (record, tile) pair: (global tile << 32) | float bits of depth;
// equal keys are ordered by record id.  Returns K = total pairs.  When keys
// is non-NULL and K <= cap, writes the sorted keys/ids and the per-tile
// [start, end) ranges ([total_tiles][2], empty tiles [0, 0)).
int64_t orc_bin(int32_t V, int64_t n, const OrcCamera* cams, const OrcOpts* o, const float* u, const float* v,
                const float* depth, const int32_t* radius, const int32_t* valid, uint32_t* tiles_touched,
                uint64_t* keys, uint32_t* ids, int64_t cap, uint32_t* ranges) {
  int64_t total_tiles = 0;
  std::vector<ViewGeom> vt = view_table(V, cams, *o, &total_tiles, nullptr);
  const float inv_tw = 1.0f / (float)o->tile_w, inv_th = 1.0f / (float)o->tile_h;
  std::vector<int32_t> rect(4 * (size_t)V * n, 0);
  int64_t K = 0;
  for (int32_t vi = 0; vi < V; ++vi) {
    const ViewGeom& g = vt[vi];
    for (int64_t i = 0; i < n; ++i) {
      const int64_t rec = (int64_t)vi * n + i;
      tiles_touched[rec] = 0;
      if (!valid[rec]) continue;
      volatile float uf = u[rec], vf = v[rec], rf = (float)radius[rec];
      volatile float xl = uf - rf, xh = uf + rf, yl = vf - rf, yh = vf + rf;
      float x0 = std::floor(xl * inv_tw), x1 = std::floor(xh * inv_tw);
      float y0 = std::floor(yl * inv_th), y1 = std::floor(yh * inv_th);
      x0 = std::max(x0, 0.0f);
      y0 = std::max(y0, 0.0f);
      x1 = std::min(x1, (float)(g.TX - 1));
      y1 = std::min(y1, (float)(g.TY - 1));
      if (!(x1 >= x0) || !(y1 >= y0)) continue;
      int32_t* rr = &rect[4 * rec];
      rr[0] = (int32_t)x0, rr[1] = (int32_t)x1, rr[2] = (int32_t)y0, rr[3] = (int32_t)y1;
      const int64_t cnt = (int64_t)(rr[1] - rr[0] + 1) * (rr[3] - rr[2] + 1);
      tiles_touched[rec] = (uint32_t)cnt;
      K += cnt;
    }
  }
  if (!keys || K > cap) return K;
  struct Ent {
    uint64_t key;
    uint32_t rec;
  };
  std::vector<Ent> e;
  e.reserve(K);
  for (int32_t vi = 0; vi < V; ++vi) {
    const ViewGeom& g = vt[vi];
    for (int64_t i = 0; i < n; ++i) {
      const int64_t rec = (int64_t)vi * n + i;
      if (!tiles_touched[rec]) continue;
      const int32_t* rr = &rect[4 * rec];
      float df = depth[rec];
      uint32_t dbits;
      std::memcpy(&dbits, &df, 4);
      for (int ty = rr[2]; ty <= rr[3]; ++ty)
        for (int tx = rr[0]; tx <= rr[1]; ++tx) {
          uint64_t gt = (uint64_t)(g.tile_off + (int64_t)ty * g.TX + tx);
          e.push_back(Ent{(gt << 32) | dbits, (uint32_t)rec});
        }
    }
  }
  std::sort(e.begin(), e.end(), [](const Ent& a, const Ent& b) {
    return a.key != b.key ? a.key < b.key : a.rec < b.rec;
  });
  for (int64_t t = 0; t < total_tiles; ++t) ranges[2 * t] = ranges[2 * t + 1] = 0;
  for (int64_t j = 0; j < K; ++j) {
    keys[j] = e[j].key;
    ids[j] = e[j].rec;
    const uint64_t t = e[j].key >> 32;
    if (j == 0 || (e[j - 1].key >> 32) != t) ranges[2 * t] = (uint32_t)j;
    if (j == K - 1 || (e[j + 1].key >> 32) != t) ranges[2 * t + 1] = (uint32_t)(j + 1);
  }
  return K;
}

// Front-to-back compositing (Eq. 2) of every pixel of V views.  Per-record
// splat data (uv [.][2], conic [.][3], opacity, rgb [.][3], radius) is indexed
// by the ids of the sorted lists.  Outputs: image (per view [3][H][W] planar,
// views concatenated), T_final and last_contrib (per view [H][W]; last_contrib
// counts the list entries up to and including the last composited one).
// Optional: eps[7] = the near-threshold windows of walk_pixel, with per-pixel
// flags (1 square edge, 2 alpha skip, 4 termination, 8 alpha cap, 16 near a
// record whose radius is near an integer, given by rec_flags bit 1 per
// record, 32 near-equal depths; rec_flags, rec_win and depth may be NULL),
// and a per-pixel hash of all decisions taken.  tile_mask (per global tile,
// may be NULL) restricts the work to the tiles marked 1; pixels of other
// tiles are left untouched.
void orc_composite_fwd(int32_t V, int64_t n, const OrcCamera* cams, const OrcOpts* o, const double* uv,
                       const double* conic, const double* opacity, const double* rgb, const int32_t* radius,
                       const uint32_t* ids, const uint32_t* ranges, double* image, double* T_final,
                       int32_t* last_contrib, const double* eps, uint8_t* flags, uint64_t* hash,
                       const uint8_t* tile_mask, const uint8_t* rec_flags, const double* rec_win,
                       const double* depth) {
  const FlagInputs fi{eps, rec_flags, rec_win, depth};
  (void)n;
  int64_t total_tiles = 0;
  std::vector<ViewGeom> vt = view_table(V, cams, *o, &total_tiles, nullptr);
  std::vector<int32_t> tile_view(total_tiles);
  for (int v = 0; v < V; ++v)
    for (int64_t t = 0; t < (int64_t)vt[v].TX * vt[v].TY; ++t) tile_view[vt[v].tile_off + t] = v;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t gt = 0; gt < total_tiles; ++gt) {
    if (tile_mask && !tile_mask[gt]) continue;
    const int vi = tile_view[gt];
    const ViewGeom& g = vt[vi];
    const int64_t lt = gt - g.tile_off;
    const int tx = (int)(lt % g.TX), ty = (int)(lt / g.TX);
    const int64_t start = ranges[2 * gt], end = ranges[2 * gt + 1];
    const int64_t plane = (int64_t)g.W * g.H;
    for (int yy = ty * o->tile_h; yy < std::min(g.H, (ty + 1) * o->tile_h); ++yy)
      for (int xx = tx * o->tile_w; xx < std::min(g.W, (tx + 1) * o->tile_w); ++xx) {
        WalkResult r =
            walk_pixel(xx + 0.5, yy + 0.5, start, end, ids, uv, conic, opacity, rgb, radius, fi, nullptr);
        const int64_t p = (int64_t)yy * g.W + xx;
        for (int ch = 0; ch < 3; ++ch) image[3 * g.pix_off + ch * plane + p] = r.C[ch] + r.T * o->bg[ch];
        T_final[g.pix_off + p] = r.T;
        last_contrib[g.pix_off + p] = r.last;
        if (flags) flags[g.pix_off + p] = r.flags;
        if (hash) hash[g.pix_off + p] = r.hash;
      }
  }
}

// Number of pixels where each record is composited (the ray hits of the
// significance score, Eq. 4): walks every pixel like orc_composite_fwd and
// counts the records in its composited list.  hits: [V*n], zeroed here.
// Pixels where a decision lies within eps of its threshold (the flags of
// orc_composite_fwd) add one to `uncertain` of every record of their tile's
// list: a single-precision walk may decide differently there.
void orc_hits(int32_t V, int64_t n, const OrcCamera* cams, const OrcOpts* o, const double* uv, const double* conic,
              const double* opacity, const double* rgb, const int32_t* radius, const uint32_t* ids,
              const uint32_t* ranges, const double* eps, uint32_t* hits, uint32_t* uncertain) {
  int64_t total_tiles = 0;
  std::vector<ViewGeom> vt = view_table(V, cams, *o, &total_tiles, nullptr);
  std::vector<int32_t> tile_view(total_tiles);
  for (int v = 0; v < V; ++v)
    for (int64_t t = 0; t < (int64_t)vt[v].TX * vt[v].TY; ++t) tile_view[vt[v].tile_off + t] = v;
  for (int64_t r = 0; r < (int64_t)V * n; ++r) {
    hits[r] = 0;
    if (uncertain) uncertain[r] = 0;
  }
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t gt = 0; gt < total_tiles; ++gt) {
    const int vi = tile_view[gt];
    const ViewGeom& g = vt[vi];
    const int64_t lt = gt - g.tile_off;
    const int tx = (int)(lt % g.TX), ty = (int)(lt / g.TX);
    const int64_t start = ranges[2 * gt], end = ranges[2 * gt + 1];
    std::vector<Contrib> list;
    for (int yy = ty * o->tile_h; yy < std::min(g.H, (ty + 1) * o->tile_h); ++yy)
      for (int xx = tx * o->tile_w; xx < std::min(g.W, (tx + 1) * o->tile_w); ++xx) {
        list.clear();
        WalkResult r =
            walk_pixel(xx + 0.5, yy + 0.5, start, end, ids, uv, conic, opacity, rgb, radius, FlagInputs{eps, nullptr, nullptr, nullptr}, &list);
        if (r.flags && uncertain) {
          // a near-threshold pixel: a walk in other arithmetic may count any record of the tile
          for (int64_t k = start; k < end; ++k) {
#pragma omp atomic
            uncertain[ids[k]] += 1u;
          }
        }
        for (const Contrib& c : list) {
#pragma omp atomic
          hits[c.rec] += 1u;
        }
      }
  }
}

// Gradient of sum(dL_dimage * image) with respect to the per-record splat
// values, written to grad_rec [V*n][9] as (u, v, A, B, C, o', r, g, b).
// Per pixel, with T_i the transmittance in front of composited Gaussian i and
// R_i = sum_{j>i} c_j a_j T_j + T_final bg (the colour behind it):
//   dC/dc_i = a_i T_i,   dC/da_i = T_i c_i - R_i / (1 - a_i);
// a = min(0.99, o' G), G = exp(-q/2): capped alphas pass no gradient.
// tile_mask as in orc_composite_fwd (pixels of other tiles contribute nothing).
void orc_composite_bwd(int32_t V, int64_t n, const OrcCamera* cams, const OrcOpts* o, const double* uv,
                       const double* conic, const double* opacity, const double* rgb, const int32_t* radius,
                       const uint32_t* ids, const uint32_t* ranges, const double* dL_dimage, double* grad_rec,
                       const uint8_t* tile_mask) {
  int64_t total_tiles = 0;
  std::vector<ViewGeom> vt = view_table(V, cams, *o, &total_tiles, nullptr);
  std::vector<int32_t> tile_view(total_tiles);
  for (int v = 0; v < V; ++v)
    for (int64_t t = 0; t < (int64_t)vt[v].TX * vt[v].TY; ++t) tile_view[vt[v].tile_off + t] = v;
  const int64_t K = total_tiles ? (int64_t)ranges[2 * (total_tiles - 1) + 1] : 0;
  int64_t Kmax = 0;
  for (int64_t t = 0; t < total_tiles; ++t) Kmax = std::max<int64_t>(Kmax, ranges[2 * t + 1]);
  (void)K;
  std::vector<double> eg((size_t)Kmax * 9, 0.0);  // per list entry; each entry belongs to one tile
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t gt = 0; gt < total_tiles; ++gt) {
    if (tile_mask && !tile_mask[gt]) continue;
    const int vi = tile_view[gt];
    const ViewGeom& g = vt[vi];
    const int64_t lt = gt - g.tile_off;
    const int tx = (int)(lt % g.TX), ty = (int)(lt / g.TX);
    const int64_t start = ranges[2 * gt], end = ranges[2 * gt + 1];
    const int64_t plane = (int64_t)g.W * g.H;
    std::vector<Contrib> list;
    for (int yy = ty * o->tile_h; yy < std::min(g.H, (ty + 1) * o->tile_h); ++yy)
      for (int xx = tx * o->tile_w; xx < std::min(g.W, (tx + 1) * o->tile_w); ++xx) {
        list.clear();
        WalkResult r =
            walk_pixel(xx + 0.5, yy + 0.5, start, end, ids, uv, conic, opacity, rgb, radius, FlagInputs{}, &list);
        const int64_t p = (int64_t)yy * g.W + xx;
        double dLdC[3], R[3];
        for (int ch = 0; ch < 3; ++ch) {
          dLdC[ch] = dL_dimage[3 * g.pix_off + ch * plane + p];
          R[ch] = r.T * o->bg[ch];
        }
        for (int64_t k = (int64_t)list.size() - 1; k >= 0; --k) {
          const Contrib& c = list[k];
          const double* col = &rgb[3 * c.rec];
          double* G9 = &eg[9 * c.entry];
          double dLda = 0.0;
          for (int ch = 0; ch < 3; ++ch) {
            G9[6 + ch] += c.alpha * c.T * dLdC[ch];
            dLda += dLdC[ch] * (c.T * col[ch] - R[ch] / (1.0 - c.alpha));
          }
          for (int ch = 0; ch < 3; ++ch) R[ch] += col[ch] * c.alpha * c.T;
          if (c.clamped) continue;
          const double A = conic[3 * c.rec], B = conic[3 * c.rec + 1], Cc = conic[3 * c.rec + 2];
          const double dLdq = -0.5 * c.alpha * dLda;
          G9[5] += c.G * dLda;
          G9[2] += dLdq * c.dx * c.dx;
          G9[3] += dLdq * 2.0 * c.dx * c.dy;
          G9[4] += dLdq * c.dy * c.dy;
          // dx = px - u, so dq/du = -(2A dx + 2B dy)
          G9[0] += dLdq * (-2.0 * (A * c.dx + B * c.dy));
          G9[1] += dLdq * (-2.0 * (B * c.dx + Cc * c.dy));
        }
      }
  }
  std::memset(grad_rec, 0, sizeof(double) * 9 * (size_t)V * n);
  for (int64_t j = 0; j < Kmax; ++j)
    for (int c = 0; c < 9; ++c) grad_rec[9 * (size_t)ids[j] + c] += eg[9 * j + c];
}

// Chain rule from per-record splat gradients of one view (grad_rec [n][9]) to
// the raw Gaussian parameters, accumulated into `out`.  Each Gaussian's
// geometry (12 inputs) and colour (54 inputs) are re-evaluated in forward-mode
// dual numbers, so this is the exact derivative of orc_project, including the
// straight-through derivative of the hard masks.
void orc_project_bwd(const OrcGaussians* g, const OrcCamera* cam, const OrcOpts* o, const double* grad_rec,
                     OrcGrads* out) {
  const int64_t n = g->n;
  const int deg = g->sh_degree;
  const int K = (deg + 1) * (deg + 1);
  double campos[3];
  campos_of(*cam, campos);
  const OrcOpts ov = view_opts(*o, *cam, n);
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t i = 0; i < n; ++i) {
    const double* gr = &grad_rec[9 * i];
    bool any = false;
    for (int c = 0; c < 9; ++c) any = any || gr[c] != 0.0;
    if (!any || !finite_inputs(*g, i)) continue;
    // geometry: inputs 0-2 mean, 3-5 log-scale, 6-9 quaternion, 10 opacity logit, 11 mask logit
    typedef Dual<12> DG;
    DG mu[3], ls[3], q[4], ol, ml;
    for (int k = 0; k < 3; ++k) mu[k] = DG::var(g->means[k * n + i], k);
    for (int k = 0; k < 3; ++k) ls[k] = DG::var(g->log_scales[k * n + i], 3 + k);
    for (int k = 0; k < 4; ++k) q[k] = DG::var(g->quats[k * n + i], 6 + k);
    ol = DG::var(g->opacity_logits[i], 10);
    if (g->mask_logits) ml = DG::var(g->mask_logits[i], 11);
    Geom<DG> ge;
    if (!project_geom<DG>(mu, ls, q, ol, g->mask_logits ? &ml : nullptr, g->mask_eps, *cam, ov, &ge)) continue;
    double dgeo[12] = {0};
    const DG* outs[6] = {&ge.u, &ge.v, &ge.A, &ge.B, &ge.C, &ge.op};
    for (int c = 0; c < 6; ++c)
      for (int k = 0; k < 12; ++k) dgeo[k] += gr[c] * outs[c]->d[k];
    // colour: inputs 0-2 mean, 3-5 diffuse, 6-50 SH rest ((k-1)*3 + ch), 51-53 band-mask logits
    typedef Dual<54> DC;
    DC cmu[3], dc[3], rest[15][3], bm[3], rgbd[3];
    for (int k = 0; k < 3; ++k) cmu[k] = DC::var(g->means[k * n + i], k);
    for (int c = 0; c < 3; ++c) dc[c] = DC::var(g->sh_dc[c * n + i], 3 + c);
    for (int k = 1; k < K; ++k)
      for (int c = 0; c < 3; ++c) rest[k - 1][c] = DC::var(g->sh_rest[((k - 1) * 3 + c) * n + i], 6 + (k - 1) * 3 + c);
    if (g->sh_mask_logits)
      for (int l = 0; l < 3; ++l) bm[l] = DC::var(g->sh_mask_logits[l * n + i], 51 + l);
    colour<DC>(cmu, dc, rest, g->sh_mask_logits ? bm : nullptr, g->sh_mask_eps, deg, campos, rgbd);
    double dcol[54] = {0};
    for (int c = 0; c < 3; ++c)
      for (int k = 0; k < 54; ++k) dcol[k] += gr[6 + c] * rgbd[c].d[k];
    // each Gaussian is owned by one loop iteration: plain accumulation
    if (out->means)
      for (int k = 0; k < 3; ++k) out->means[k * n + i] += dgeo[k] + dcol[k];
    if (out->log_scales)
      for (int k = 0; k < 3; ++k) out->log_scales[k * n + i] += dgeo[3 + k];
    if (out->quats)
      for (int k = 0; k < 4; ++k) out->quats[k * n + i] += dgeo[6 + k];
    if (out->opacity_logits) out->opacity_logits[i] += dgeo[10];
    if (out->mask_logits && g->mask_logits) out->mask_logits[i] += dgeo[11];
    if (out->sh_dc)
      for (int c = 0; c < 3; ++c) out->sh_dc[c * n + i] += dcol[3 + c];
    if (out->sh_rest)
      for (int k = 1; k < K; ++k)
        for (int c = 0; c < 3; ++c) out->sh_rest[((k - 1) * 3 + c) * n + i] += dcol[6 + (k - 1) * 3 + c];
    if (out->sh_mask_logits && g->sh_mask_logits)
      for (int l = 0; l < 3; ++l) out->sh_mask_logits[l * n + i] += dcol[51 + l];
  }
}

}  // extern "C"
