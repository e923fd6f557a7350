// Per-tile front-to-back compositing (Eq. 2) and its backward.
//
// One workgroup per tile (global tile ids span all views of the call).  The
// tile's sorted list is walked in batches of up to 256 splat records that the
// workgroup gathers into LDS; every lane then walks the batch for its
// pixel(s), reading each record as a wave-uniform LDS broadcast.  No MFMA:
// the work per (pixel, splat) pair is ~20 VALU operations and one exp.
//
// Forward: lanes whose pixels have terminated drop out of the walk through
// the exec mask; before each batch the waves vote and the whole workgroup
// leaves once every pixel is done.
//
// Backward: the list is re-walked back to front from the tile's largest
// last_contrib; each pixel recovers the transmittance in front of a splat by
// dividing by (1 - alpha) and carries the dL/dC-weighted colour behind it, so
// no per-pixel list is stored.  Per-pair partials (9 floats) are summed over
// the lane's pixels, over the wave (DPP), and over the workgroup (LDS float
// atomics), then one global atomic per non-zero attribute per (tile, splat).
#include "gs_common.h"
#include "kernels.h"

namespace gs {

struct TileCtx {
  int view;
  int tx, ty;
  uint32_t start, end;
};

__device__ __forceinline__ TileCtx tile_ctx(const ViewTable& vt, const RenderArgs& a, int gtile) {
  TileCtx c;
  c.view = view_of_tile(vt, gtile);
  const ViewArgs& va = vt.v[c.view];
  const int lt = gtile - va.tile_off;
  c.ty = lt / va.TX;
  c.tx = lt - c.ty * va.TX;
  c.start = 0;
  c.end = 0;
  if (*a.status == 0) {
    c.start = a.ranges[2 * gtile];
    c.end = a.ranges[2 * gtile + 1];
  }
  return c;
}

template <int PPT>
__global__ __launch_bounds__(256) void render_fwd_kernel(RenderArgs a, ViewTable vt, float* __restrict__ image,
                                                         float* __restrict__ T_final, int32_t* __restrict__ last_out) {
  __shared__ float4 s_a[GS_MAX_BATCH], s_b[GS_MAX_BATCH], s_c[GS_MAX_BATCH];
  __shared__ int s_alive[16];
  const int gtile = blockIdx.x;
  const TileCtx tc = tile_ctx(vt, a, gtile);
  const ViewArgs& va = vt.v[tc.view];
  const int nthreads = blockDim.x;
  const int tw = 1 << a.log2_tw;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave, nwaves = nthreads / kWave;

  float px[PPT], py[PPT], T[PPT], C0[PPT], C1[PPT], C2[PPT];
  int last[PPT];
  bool done[PPT];
#pragma unroll
  for (int p = 0; p < PPT; ++p) {
    const int li = threadIdx.x * PPT + p;
    const int x = tc.tx * tw + (li & (tw - 1));
    const int y = (tc.ty << a.log2_th) + (li >> a.log2_tw);
    px[p] = (float)x + 0.5f;
    py[p] = (float)y + 0.5f;
    T[p] = 1.0f;
    C0[p] = C1[p] = C2[p] = 0.0f;
    last[p] = 0;
    done[p] = !(x < va.W && y < va.H);
  }

  for (uint32_t bs = tc.start; bs < tc.end; bs += a.batch) {
    bool alive = false;
#pragma unroll
    for (int p = 0; p < PPT; ++p) alive |= !done[p];
    const uint64_t vote = __ballot(alive);
    if (lane == 0) s_alive[wave] = vote != 0;
    __syncthreads();
    int any = 0;
    for (int w = 0; w < nwaves; ++w) any |= s_alive[w];
    if (!any) break;
    const int cnt = (int)min((uint32_t)a.batch, tc.end - bs);
    for (int i = threadIdx.x; i < cnt; i += nthreads) {
      const uint32_t rec = a.ids[bs + i];
      s_a[i] = a.splats[(size_t)rec * 3 + 0];
      s_b[i] = a.splats[(size_t)rec * 3 + 1];
      s_c[i] = a.splats[(size_t)rec * 3 + 2];
    }
    __syncthreads();
    for (int j = 0; j < cnt; ++j) {
      const float4 ra = s_a[j], rb = s_b[j];
#pragma unroll
      for (int p = 0; p < PPT; ++p) {
        if (done[p]) continue;
        Eval e;
        if (!eval_splat(px[p], py[p], ra.x, ra.y, ra.z, ra.w, rb.x, rb.y, rb.z, &e)) continue;
        if (e.alpha < kAlphaMin) continue;
        const float Tn = T[p] * (1.0f - e.alpha);
        if (Tn < kTMin) {
          done[p] = true;
          continue;
        }
        const float4 rc = s_c[j];
        const float w = e.alpha * T[p];
        C0[p] += rc.x * w;
        C1[p] += rc.y * w;
        C2[p] += rc.z * w;
        T[p] = Tn;
        last[p] = (int)(bs + j - tc.start) + 1;
      }
    }
  }

  const int64_t plane = (int64_t)va.W * va.H;
#pragma unroll
  for (int p = 0; p < PPT; ++p) {
    const int x = (int)px[p], y = (int)py[p];
    if (x < va.W && y < va.H) {
      const int64_t pix = (int64_t)y * va.W + x;
      float* img = image + 3 * (int64_t)va.pix_off;
      img[pix] = C0[p] + T[p] * a.bg[0];
      img[plane + pix] = C1[p] + T[p] * a.bg[1];
      img[2 * plane + pix] = C2[p] + T[p] * a.bg[2];
      T_final[va.pix_off + pix] = T[p];
      last_out[va.pix_off + pix] = last[p];
    }
  }
}

template <int PPT>
__global__ __launch_bounds__(256) void render_bwd_kernel(RenderArgs a, ViewTable vt, const float* __restrict__ T_final,
                                                         const int32_t* __restrict__ last_in,
                                                         const float* __restrict__ dL_dimage,
                                                         float* __restrict__ grad_rec) {
  __shared__ float4 s_a[GS_MAX_BATCH], s_b[GS_MAX_BATCH], s_c[GS_MAX_BATCH];
  __shared__ uint32_t s_id[GS_MAX_BATCH];
  __shared__ float s_acc[GS_MAX_BATCH * GS_GRAD_FLOATS];
  __shared__ int s_max[16];
  const int gtile = blockIdx.x;
  const TileCtx tc = tile_ctx(vt, a, gtile);
  const ViewArgs& va = vt.v[tc.view];
  const int nthreads = blockDim.x;
  const int tw = 1 << a.log2_tw;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave, nwaves = nthreads / kWave;
  const int64_t plane = (int64_t)va.W * va.H;

  float px[PPT], py[PPT], T[PPT], g0[PPT], g1[PPT], g2[PPT], RdL[PPT];
  int lc[PPT];
  int my_max = 0;
#pragma unroll
  for (int p = 0; p < PPT; ++p) {
    const int li = threadIdx.x * PPT + p;
    const int x = tc.tx * tw + (li & (tw - 1));
    const int y = (tc.ty << a.log2_th) + (li >> a.log2_tw);
    px[p] = (float)x + 0.5f;
    py[p] = (float)y + 0.5f;
    T[p] = 1.0f;
    g0[p] = g1[p] = g2[p] = RdL[p] = 0.0f;
    lc[p] = 0;
    if (x < va.W && y < va.H) {
      const int64_t pix = (int64_t)y * va.W + x;
      const float* dl = dL_dimage + 3 * (int64_t)va.pix_off;
      T[p] = T_final[va.pix_off + pix];
      lc[p] = last_in[va.pix_off + pix];
      g0[p] = dl[pix];
      g1[p] = dl[plane + pix];
      g2[p] = dl[2 * plane + pix];
      RdL[p] = T[p] * (a.bg[0] * g0[p] + a.bg[1] * g1[p] + a.bg[2] * g2[p]);
      my_max = max(my_max, lc[p]);
    }
  }
  // workgroup max of last_contrib
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) my_max = max(my_max, __shfl_xor(my_max, o, kWave));
  if (lane == 0) s_max[wave] = my_max;
  __syncthreads();
  int maxlast = 0;
  for (int w = 0; w < nwaves; ++w) maxlast = max(maxlast, s_max[w]);
  maxlast = min(maxlast, (int)(tc.end - tc.start));  // never walk past the tile's list

  const uint32_t wend = tc.start + (uint32_t)maxlast;
  for (uint32_t be = wend; be > tc.start;) {
    const uint32_t bs = (be - tc.start > (uint32_t)a.batch) ? be - a.batch : tc.start;
    const int cnt = (int)(be - bs);
    for (int i = threadIdx.x; i < cnt; i += nthreads) {
      const uint32_t rec = a.ids[bs + i];
      s_id[i] = rec;
      s_a[i] = a.splats[(size_t)rec * 3 + 0];
      s_b[i] = a.splats[(size_t)rec * 3 + 1];
      s_c[i] = a.splats[(size_t)rec * 3 + 2];
    }
    for (int i = threadIdx.x; i < cnt * GS_GRAD_FLOATS; i += nthreads) s_acc[i] = 0.0f;
    __syncthreads();
    for (int j = cnt - 1; j >= 0; --j) {
      const int jr = (int)(bs - tc.start) + j;  // index within the tile's list
      const float4 ra = s_a[j], rb = s_b[j], rc = s_c[j];
      float gu = 0.f, gv = 0.f, gA = 0.f, gB = 0.f, gC = 0.f, go = 0.f, gr = 0.f, gg = 0.f, gb = 0.f;
      bool any = false;
#pragma unroll
      for (int p = 0; p < PPT; ++p) {
        if (jr >= lc[p]) continue;
        Eval e;
        if (!eval_splat(px[p], py[p], ra.x, ra.y, ra.z, ra.w, rb.x, rb.y, rb.z, &e)) continue;
        if (e.alpha < kAlphaMin) continue;
        any = true;
        const float inv = __builtin_amdgcn_rcpf(1.0f - e.alpha);
        T[p] *= inv;  // transmittance in front of this splat
        const float wgt = e.alpha * T[p];
        gr += wgt * g0[p];
        gg += wgt * g1[p];
        gb += wgt * g2[p];
        const float cd = rc.x * g0[p] + rc.y * g1[p] + rc.z * g2[p];
        const float dLda = T[p] * cd - RdL[p] * inv;
        RdL[p] += cd * wgt;
        if (!(e.raw > kAlphaMax)) {
          go += e.G * dLda;
          const float dLdq = -0.5f * e.alpha * dLda;
          gA += dLdq * e.dx * e.dx;
          gB += dLdq * 2.0f * e.dx * e.dy;
          gC += dLdq * e.dy * e.dy;
          gu += -2.0f * dLdq * (ra.z * e.dx + ra.w * e.dy);
          gv += -2.0f * dLdq * (ra.w * e.dx + rb.x * e.dy);
        }
      }
      if (__ballot(any) != 0) {
        gu = wave_sum_lane63(gu);
        gv = wave_sum_lane63(gv);
        gA = wave_sum_lane63(gA);
        gB = wave_sum_lane63(gB);
        gC = wave_sum_lane63(gC);
        go = wave_sum_lane63(go);
        gr = wave_sum_lane63(gr);
        gg = wave_sum_lane63(gg);
        gb = wave_sum_lane63(gb);
        if (lane == kWave - 1) {
          float* acc = &s_acc[j * GS_GRAD_FLOATS];
          atomicAdd(acc + 0, gu);
          atomicAdd(acc + 1, gv);
          atomicAdd(acc + 2, gA);
          atomicAdd(acc + 3, gB);
          atomicAdd(acc + 4, gC);
          atomicAdd(acc + 5, go);
          atomicAdd(acc + 6, gr);
          atomicAdd(acc + 7, gg);
          atomicAdd(acc + 8, gb);
        }
      }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < cnt * GS_GRAD_FLOATS; i += nthreads) {
      const float val = s_acc[i];
      if (val != 0.0f) {
        const int e = i / GS_GRAD_FLOATS;
        unsafeAtomicAdd(&grad_rec[(size_t)s_id[e] * GS_GRAD_FLOATS + (i - e * GS_GRAD_FLOATS)], val);
      }
    }
    __syncthreads();
    be = bs;
  }
}

static int tile_threads(const RenderArgs& a) { return (1 << (a.log2_tw + a.log2_th)) / a.ppt; }

hipError_t launch_render_fwd(const RenderArgs& a, const ViewTable& vt, float* image, float* T_final,
                             int32_t* last_contrib, hipStream_t s) {
  if (vt.total_tiles == 0) return hipSuccess;
  const dim3 grid((unsigned)vt.total_tiles), block((unsigned)tile_threads(a));
  switch (a.ppt) {
    case 1: hipLaunchKernelGGL(render_fwd_kernel<1>, grid, block, 0, s, a, vt, image, T_final, last_contrib); break;
    case 2: hipLaunchKernelGGL(render_fwd_kernel<2>, grid, block, 0, s, a, vt, image, T_final, last_contrib); break;
    default: hipLaunchKernelGGL(render_fwd_kernel<4>, grid, block, 0, s, a, vt, image, T_final, last_contrib); break;
  }
  return hipGetLastError();
}

hipError_t launch_render_bwd(const RenderArgs& a, const ViewTable& vt, const float* T_final,
                             const int32_t* last_contrib, const float* dL_dimage, float* grad_rec, hipStream_t s) {
  if (vt.total_tiles == 0) return hipSuccess;
  const dim3 grid((unsigned)vt.total_tiles), block((unsigned)tile_threads(a));
  switch (a.ppt) {
    case 1:
      hipLaunchKernelGGL(render_bwd_kernel<1>, grid, block, 0, s, a, vt, T_final, last_contrib, dL_dimage, grad_rec);
      break;
    case 2:
      hipLaunchKernelGGL(render_bwd_kernel<2>, grid, block, 0, s, a, vt, T_final, last_contrib, dL_dimage, grad_rec);
      break;
    default:
      hipLaunchKernelGGL(render_bwd_kernel<4>, grid, block, 0, s, a, vt, T_final, last_contrib, dL_dimage, grad_rec);
      break;
  }
  return hipGetLastError();
}

}  // namespace gs
