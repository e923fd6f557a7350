// Backward of the projection: per-record splat gradients (u, v, A, B, C, o',
// r, g, b) -> raw Gaussian parameters, accumulated over the V views of the
// call (one thread per Gaussian, so no atomics), then added (+=) to the
// caller's gradient arrays.  Straight-through estimator for the hard masks
// (Eq. 3, Eq. 5): d(mask)/d(logit) = sigmoid'(logit).
//
// Chain, per view (Sigma' = T Sigma T^T + sI, T = J W, Q = Sigma'^-1 = conic):
//   dL/dSigma'  = -Q G_Q Q              (G_Q symmetric: [[gA, gB/2], [gB/2, gC]])
//   dL/dSigma   = T^T dL/dSigma' T,     dL/dT = 2 dL/dSigma' T Sigma
//   dL/dJ       = dL/dT W^T  -> camera-space mean t (through J's entries and
//                 the clamp of the lateral ratios), plus the screen mean (u, v)
//   dL/dmu      = W^T dL/dt  + view-direction term of the SH colour
//   dL/dM       = 2 dL/dSigma M  with M = Rq diag(s) -> scales and rotation,
//                 then through the quaternion normalisation.
#include "gs_common.h"
#include "kernels.h"

namespace gs {

// Gradient of the 15 SH basis polynomials (k = 1..15) w.r.t. (x, y, z),
// contracted with per-function weights w[k-1]: returns sum_k w_k grad Y_k.
__device__ __forceinline__ void sh_grad15(float x, float y, float z, const float w[15], float* gx, float* gy,
                                          float* gz) {
  const float xx = x * x, yy = y * y, zz = z * z;
  float ax = 0.f, ay = 0.f, az = 0.f;
  // band 1
  ay += -kC1 * w[0];
  az += kC1 * w[1];
  ax += -kC1 * w[2];
  // band 2
  ax += kC2a * y * w[3];
  ay += kC2a * x * w[3];
  ay += -kC2a * z * w[4];
  az += -kC2a * y * w[4];
  ax += -2.f * kC2b * x * w[5];
  ay += -2.f * kC2b * y * w[5];
  az += 4.f * kC2b * z * w[5];
  ax += -kC2a * z * w[6];
  az += -kC2a * x * w[6];
  ax += 2.f * kC2c * x * w[7];
  ay += -2.f * kC2c * y * w[7];
  // band 3
  ax += -6.f * kC3a * x * y * w[8];
  ay += -kC3a * (3.f * xx - 3.f * yy) * w[8];
  ax += kC3b * y * z * w[9];
  ay += kC3b * x * z * w[9];
  az += kC3b * x * y * w[9];
  ax += 2.f * kC3c * x * y * w[10];
  ay += -kC3c * (4.f * zz - xx - 3.f * yy) * w[10];
  az += -8.f * kC3c * y * z * w[10];
  ax += -6.f * kC3d * x * z * w[11];
  ay += -6.f * kC3d * y * z * w[11];
  az += kC3d * (6.f * zz - 3.f * xx - 3.f * yy) * w[11];
  ax += -kC3c * (4.f * zz - 3.f * xx - yy) * w[12];
  ay += 2.f * kC3c * x * y * w[12];
  az += -8.f * kC3c * x * z * w[12];
  ax += 2.f * kC3e * x * z * w[13];
  ay += -2.f * kC3e * y * z * w[13];
  az += kC3e * (xx - yy) * w[13];
  ax += -kC3a * (3.f * xx - 3.f * yy) * w[14];
  ay += 6.f * kC3a * x * y * w[14];
  *gx = ax;
  *gy = ay;
  *gz = az;
}

template <int DEG>
__global__ __launch_bounds__(256) void project_bwd_kernel(ProjectBwdArgs b, ViewTable vt) {
  const ProjectArgs& a = b.p;
  const int64_t n = a.n;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int V = vt.nviews;

  // Skip Gaussians that received no splat gradient in any view.
  bool any = false;
  for (int v = 0; v < V && !any; ++v) {
    const float* g = b.grad_rec + ((size_t)v * n + i) * GS_GRAD_FLOATS;
#pragma unroll
    for (int k = 0; k < GS_GRAD_FLOATS; ++k) any |= g[k] != 0.0f;
  }
  if (!any) return;  // culled records never receive splat gradients

  float mu[3], ls[3], q[4], dc[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    mu[k] = a.means[k * n + i];
    ls[k] = a.log_scales[k * n + i];
    dc[k] = a.sh_dc[k * n + i];
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) q[k] = a.quats[k * n + i];
  const float ol = a.opacity_logits[i];
  constexpr int NR = DEG > 0 ? (DEG + 1) * (DEG + 1) - 1 : 1;
  float rest[NR][3];
  float bm[3] = {0.f, 0.f, 0.f};
  bool band_on[4] = {true, true, true, true};
  if (DEG > 0) {
    if (a.sh_mask_logits) {
#pragma unroll
      for (int l = 1; l <= 3; ++l) {
        bm[l - 1] = a.sh_mask_logits[(l - 1) * n + i];
        band_on[l] = bm[l - 1] > a.sh_mask_thr;
      }
    }
    // every band's coefficients are read: the band-mask gradient needs them
    // even when the band is off (straight-through estimator)
#pragma unroll
    for (int k = 1; k <= NR; ++k)
#pragma unroll
      for (int c = 0; c < 3; ++c) rest[k - 1][c] = a.sh_rest[((k - 1) * 3 + c) * n + i];
  }

  // forward quantities shared by all views
  const float qn = sqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  const float iq = 1.0f / qn;
  const float w = q[0] * iq, x = q[1] * iq, y = q[2] * iq, z = q[3] * iq;
  float Rq[3][3] = {{1.f - 2.f * (y * y + z * z), 2.f * (x * y - w * z), 2.f * (x * z + w * y)},
                    {2.f * (x * y + w * z), 1.f - 2.f * (x * x + z * z), 2.f * (y * z - w * x)},
                    {2.f * (x * z - w * y), 2.f * (y * z + w * x), 1.f - 2.f * (x * x + y * y)}};
  float s[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) s[k] = __expf(ls[k]);
  float M[3][3];  // Rq diag(s)
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int k = 0; k < 3; ++k) M[r][k] = Rq[r][k] * s[k];
  float Sig[3][3];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) Sig[r][c] = M[r][0] * M[c][0] + M[r][1] * M[c][1] + M[r][2] * M[c][2];
  const float op = sigmoidf(ol);

  // accumulated gradients
  float gmu[3] = {0.f, 0.f, 0.f};
  float gSig[3][3] = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}};
  float gop = 0.f;
  float gdc[3] = {0.f, 0.f, 0.f};
  float grest[NR][3];
  float gbm[3] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int k = 0; k < NR; ++k) grest[k][0] = grest[k][1] = grest[k][2] = 0.f;

  for (int v = 0; v < V; ++v) {
    const float* gr = b.grad_rec + ((size_t)v * n + i) * GS_GRAD_FLOATS;
    const float gu = gr[0], gv = gr[1], gA = gr[2], gB = gr[3], gC = gr[4], go = gr[5];
    const float grgb[3] = {gr[6], gr[7], gr[8]};
    bool nz = false;
#pragma unroll
    for (int k = 0; k < GS_GRAD_FLOATS; ++k) nz |= gr[k] != 0.0f;
    if (!nz) continue;
    const ViewArgs& c = vt.v[v];
    const float t0 = c.R[0] * mu[0] + c.R[1] * mu[1] + c.R[2] * mu[2] + c.t[0];
    const float t1 = c.R[3] * mu[0] + c.R[4] * mu[1] + c.R[5] * mu[2] + c.t[1];
    const float t2 = c.R[6] * mu[0] + c.R[7] * mu[1] + c.R[8] * mu[2] + c.t[2];
    const float iz = 1.0f / t2;
    const float ux = t0 * iz, uy = t1 * iz;
    const bool inx = ux >= -c.limx && ux <= c.limx;
    const bool iny = uy >= -c.limy && uy <= c.limy;
    const float rx = fminf(fmaxf(ux, -c.limx), c.limx);
    const float ry = fminf(fmaxf(uy, -c.limy), c.limy);
    const float j00 = c.fx * iz, j02 = -c.fx * rx * iz, j11 = c.fy * iz, j12 = -c.fy * ry * iz;
    float Tm[2][3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      Tm[0][k] = j00 * c.R[k] + j02 * c.R[6 + k];
      Tm[1][k] = j11 * c.R[3 + k] + j12 * c.R[6 + k];
    }
    float TS[2][3];  // T Sigma
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int k = 0; k < 3; ++k) TS[r][k] = Tm[r][0] * Sig[0][k] + Tm[r][1] * Sig[1][k] + Tm[r][2] * Sig[2][k];
    const float ca = TS[0][0] * Tm[0][0] + TS[0][1] * Tm[0][1] + TS[0][2] * Tm[0][2] + a.lowpass;
    const float cb = TS[0][0] * Tm[1][0] + TS[0][1] * Tm[1][1] + TS[0][2] * Tm[1][2];
    const float cc = TS[1][0] * Tm[1][0] + TS[1][1] * Tm[1][1] + TS[1][2] * Tm[1][2] + a.lowpass;
    const float idet = 1.0f / (ca * cc - cb * cb);
    const float QA = cc * idet, QB = -cb * idet, QC = ca * idet;
    // dL/dSigma' = -Q G_Q Q
    const float P00 = QA * gA + QB * 0.5f * gB, P01 = QA * 0.5f * gB + QB * gC;
    const float P10 = QB * gA + QC * 0.5f * gB, P11 = QB * 0.5f * gB + QC * gC;
    const float G00 = -(P00 * QA + P01 * QB);
    const float G01 = -(P00 * QB + P01 * QC);
    const float G11 = -(P10 * QB + P11 * QC);
    // dL/dSigma += T^T G T
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int k = 0; k < 3; ++k)
        gSig[r][k] += Tm[0][r] * (G00 * Tm[0][k] + G01 * Tm[1][k]) + Tm[1][r] * (G01 * Tm[0][k] + G11 * Tm[1][k]);
    // dL/dT = 2 G T Sigma
    float gT[2][3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      gT[0][k] = 2.f * (G00 * TS[0][k] + G01 * TS[1][k]);
      gT[1][k] = 2.f * (G01 * TS[0][k] + G11 * TS[1][k]);
    }
    // T = J W: only J00, J02, J11, J12 vary
    const float gj00 = gT[0][0] * c.R[0] + gT[0][1] * c.R[1] + gT[0][2] * c.R[2];
    const float gj02 = gT[0][0] * c.R[6] + gT[0][1] * c.R[7] + gT[0][2] * c.R[8];
    const float gj11 = gT[1][0] * c.R[3] + gT[1][1] * c.R[4] + gT[1][2] * c.R[5];
    const float gj12 = gT[1][0] * c.R[6] + gT[1][1] * c.R[7] + gT[1][2] * c.R[8];
    const float iz2 = iz * iz;
    float gt0 = gu * c.fx * iz, gt1 = gv * c.fy * iz;
    float gt2 = -gu * c.fx * t0 * iz2 - gv * c.fy * t1 * iz2;
    gt2 += -gj00 * c.fx * iz2 - gj11 * c.fy * iz2;
    // J02 = -fx rx / z with rx = clamp(x / z): d/dx = -fx/z^2 (unclamped), d/dz = fx rx/z^2 + fx x/z^3 (unclamped)
    gt2 += gj02 * c.fx * rx * iz2 + gj12 * c.fy * ry * iz2;
    if (inx) {
      gt0 += -gj02 * c.fx * iz2;
      gt2 += gj02 * c.fx * t0 * iz2 * iz;
    }
    if (iny) {
      gt1 += -gj12 * c.fy * iz2;
      gt2 += gj12 * c.fy * t1 * iz2 * iz;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) gmu[k] += c.R[k] * gt0 + c.R[3 + k] * gt1 + c.R[6 + k] * gt2;
    gop += go;
    if (b.g_mean2d) {
      b.g_mean2d[((size_t)v * 2 + 0) * n + i] += gu;
      b.g_mean2d[((size_t)v * 2 + 1) * n + i] += gv;
    }
    // colour
    float d0 = mu[0] - c.campos[0], d1 = mu[1] - c.campos[1], d2 = mu[2] - c.campos[2];
    float Y[15];
    float il = 1.0f, dx = 0.f, dy = 0.f, dz = 0.f;
    if (DEG > 0) {
      il = 1.0f / sqrtf(d0 * d0 + d1 * d1 + d2 * d2);
      dx = d0 * il, dy = d1 * il, dz = d2 * il;
      sh_basis15(dx, dy, dz, Y);
    }
    float pre[3] = {dc[0], dc[1], dc[2]};
#pragma unroll
    for (int l = 1; l <= DEG; ++l) {
      if (!band_on[l]) continue;
#pragma unroll
      for (int k = l * l; k < (l + 1) * (l + 1); ++k)
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) pre[ch] += Y[k - 1] * rest[k - 1][ch];
    }
    float gpre[3];
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
      gpre[ch] = pre[ch] < 0.f ? 0.f : grgb[ch];
      gdc[ch] += gpre[ch];
    }
    if (DEG > 0) {
      float wY[15];
#pragma unroll
      for (int k = 0; k < 15; ++k) wY[k] = 0.f;
#pragma unroll
      for (int l = 1; l <= DEG; ++l) {
        float band = 0.f;
#pragma unroll
        for (int k = l * l; k < (l + 1) * (l + 1); ++k) {
          const float cg = rest[k - 1][0] * gpre[0] + rest[k - 1][1] * gpre[1] + rest[k - 1][2] * gpre[2];
          band += Y[k - 1] * cg;
          if (band_on[l]) {
            wY[k - 1] = cg;
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) grest[k - 1][ch] += Y[k - 1] * gpre[ch];
          }
        }
        gbm[l - 1] += band;
      }
      float gdx, gdy, gdz;
      sh_grad15(dx, dy, dz, wY, &gdx, &gdy, &gdz);
      const float dot = dx * gdx + dy * gdy + dz * gdz;
      gmu[0] += (gdx - dx * dot) * il;
      gmu[1] += (gdy - dy * dot) * il;
      gmu[2] += (gdz - dz * dot) * il;
    }
  }

  // Sigma = M M^T -> dL/dM = 2 G_Sigma M (G_Sigma symmetrised)
  float gM[3][3];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      float acc = 0.f;
#pragma unroll
      for (int c2 = 0; c2 < 3; ++c2) acc += (gSig[r][c2] + gSig[c2][r]) * M[c2][k];
      gM[r][k] = acc;
    }
  float gsc[3], gR[3][3];
#pragma unroll
  for (int k = 0; k < 3; ++k) gsc[k] = gM[0][k] * Rq[0][k] + gM[1][k] * Rq[1][k] + gM[2][k] * Rq[2][k];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int k = 0; k < 3; ++k) gR[r][k] = gM[r][k] * s[k];
  const float gw = 2.f * (-z * gR[0][1] + y * gR[0][2] + z * gR[1][0] - x * gR[1][2] - y * gR[2][0] + x * gR[2][1]);
  const float gx = 2.f * (y * gR[0][1] + z * gR[0][2] + y * gR[1][0] - 2.f * x * gR[1][1] - w * gR[1][2] +
                          z * gR[2][0] + w * gR[2][1] - 2.f * x * gR[2][2]);
  const float gy = 2.f * (-2.f * y * gR[0][0] + x * gR[0][1] + w * gR[0][2] + x * gR[1][0] + z * gR[1][2] -
                          w * gR[2][0] + z * gR[2][1] - 2.f * y * gR[2][2]);
  const float gz = 2.f * (-2.f * z * gR[0][0] - w * gR[0][1] + x * gR[0][2] + w * gR[1][0] - 2.f * z * gR[1][1] +
                          y * gR[1][2] + x * gR[2][0] + y * gR[2][1]);
  const float qd = w * gw + x * gx + y * gy + z * gz;
  const float gq[4] = {(gw - w * qd) * iq, (gx - x * qd) * iq, (gy - y * qd) * iq, (gz - z * qd) * iq};

#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (b.g_means) b.g_means[k * n + i] += gmu[k];
    if (b.g_log_scales) b.g_log_scales[k * n + i] += gsc[k] * s[k];
    if (b.g_sh_dc) b.g_sh_dc[k * n + i] += gdc[k];
  }
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (b.g_quats) b.g_quats[k * n + i] += gq[k];
  if (b.g_opacity_logits) b.g_opacity_logits[i] += gop * op * (1.f - op);
  if (b.g_mask_logits && a.mask_logits) {
    // o' = M o, s' = M s (M = 1 here): dL/dM = o dL/do' + sum_k s_k dL/ds'_k
    const float sm = sigmoidf(a.mask_logits[i]);
    const float gMask = gop * op + gsc[0] * s[0] + gsc[1] * s[1] + gsc[2] * s[2];
    b.g_mask_logits[i] += gMask * sm * (1.f - sm);
  }
  if (DEG > 0) {
    if (b.g_sh_rest) {
#pragma unroll
      for (int k = 1; k <= NR; ++k)
#pragma unroll
        for (int c = 0; c < 3; ++c) b.g_sh_rest[((k - 1) * 3 + c) * n + i] += grest[k - 1][c];
    }
    if (b.g_sh_mask_logits && a.sh_mask_logits) {
#pragma unroll
      for (int l = 1; l <= DEG; ++l) {
        const float sm = sigmoidf(bm[l - 1]);
        b.g_sh_mask_logits[(l - 1) * n + i] += gbm[l - 1] * sm * (1.f - sm);
      }
    }
  }
}

hipError_t launch_project_bwd(const ProjectBwdArgs& a, const ViewTable& vt, int deg, hipStream_t s) {
  if (a.p.n == 0) return hipSuccess;
  const dim3 block(256), grid((unsigned)((a.p.n + 255) / 256));
  switch (deg) {
    case 0: hipLaunchKernelGGL(project_bwd_kernel<0>, grid, block, 0, s, a, vt); break;
    case 1: hipLaunchKernelGGL(project_bwd_kernel<1>, grid, block, 0, s, a, vt); break;
    case 2: hipLaunchKernelGGL(project_bwd_kernel<2>, grid, block, 0, s, a, vt); break;
    default: hipLaunchKernelGGL(project_bwd_kernel<3>, grid, block, 0, s, a, vt); break;
  }
  return hipGetLastError();
}

}  // namespace gs
