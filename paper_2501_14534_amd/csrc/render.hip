// Per-tile front-to-back compositing (Eq. 2) and its backward.
//
// One workgroup per tile (global tile ids span all views of the call).  The
// tile's sorted list is walked in batches of up to 256 splat records that the
// workgroup gathers into LDS; every lane then walks the batch for its
// pixel(s), reading each record as a wave-uniform LDS broadcast.  No MFMA:
// the work per (pixel, splat) pair is ~20 VALU operations and one exp.
//
// Sub-tile culling (CULL): while staging a batch, each record's conservative
// alpha >= 1/255 footprint (the ellipse q <= 2 ln(255 o') bounded by its
// square, widened by rounding margins) is tested against the pixel box of
// every wave; wave 0 then builds one ordered list of batch indices per wave,
// and each wave walks only its own list.  Culled records fail a per-pixel
// test for every pixel of that wave, so the result is unchanged.
//
// Forward: lanes whose pixels have terminated drop out of the walk through
// the exec mask; before each batch the waves vote and the whole workgroup
// leaves once every pixel is done.
//
// Backward: the list is re-walked back to front from the tile's largest
// last_contrib; each pixel recovers the transmittance in front of a splat by
// dividing by (1 - alpha) and carries the dL/dC-weighted colour behind it, so
// no per-pixel list is stored.  Per-pair partials (9 floats) are summed over
// the lane's pixels, over the wave (DPP), then over the workgroup's waves in a
// fixed order (LDS), and stored once per (tile, splat) at the pair's emission
// position: no atomics, so the result is bitwise reproducible.
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

// Pixels of a tile are split into one sub-tile per wave (as square as the
// tile allows, chosen on the host); a lane covers PPT consecutive pixels of a
// sub-tile row.  Pixel p of thread t:
__device__ __forceinline__ void pixel_of(const RenderArgs& a, int ppt, int t, int p, int tx, int ty, int* x, int* y) {
  const int w = t >> 6, l = t & (kWave - 1);
  const int sxi = w & ((1 << a.log2_sx) - 1), syi = w >> a.log2_sx;
  const int li = l * ppt + p;
  *x = (tx << a.log2_tw) + (sxi << a.log2_sw) + (li & ((1 << a.log2_sw) - 1));
  *y = (ty << a.log2_th) + (syi << a.log2_sh) + (li >> a.log2_sw);
}

// Pixel-centre box of wave w's sub-tile.
struct Box {
  float x0, x1, y0, y1;
};

__device__ __forceinline__ Box wave_box(const RenderArgs& a, int w, int tx, int ty) {
  const int sxi = w & ((1 << a.log2_sx) - 1), syi = w >> a.log2_sx;
  const int x0 = (tx << a.log2_tw) + (sxi << a.log2_sw), y0 = (ty << a.log2_th) + (syi << a.log2_sh);
  Box b;
  b.x0 = (float)x0 + 0.5f;
  b.x1 = (float)(x0 + (1 << a.log2_sw) - 1) + 0.5f;
  b.y0 = (float)y0 + 0.5f;
  b.y1 = (float)(y0 + (1 << a.log2_sh) - 1) + 0.5f;
  return b;
}

// Bit w set when record (u, v, conic, o', radius) may composite some pixel of wave w.
__device__ __forceinline__ uint32_t footprint_mask(const RenderArgs& a, float4 ra, float4 rb, int nwaves, int tx,
                                                   int ty) {
  const float u = ra.x, v = ra.y, A = ra.z, B = ra.w, C = rb.x, o = rb.y, r = rb.z;
  if (!(o >= kAlphaMin * 0.999f)) return 0u;  // alpha <= o' < 1/255 at every pixel
  float ex = r, ey = r;
  const float det = A * C - B * B;
  if (det > 0.f) {
    const float tr = 0.5f * (A + C);
    const float lmax = tr + sqrtf(fmaxf(0.f, tr * tr - det));
    if (lmax * lmax <= 1e3f * det) {  // condition number <= 1e3: rounding of q stays far below the margins
      const float qm = 2.0f * __logf(255.0f * o) * 1.002f + 0.002f;
      const float idet = 1.0f / det;
      ex = fminf(r, sqrtf(fmaxf(qm, 0.f) * C * idet) * 1.001f + 0.01f);
      ey = fminf(r, sqrtf(fmaxf(qm, 0.f) * A * idet) * 1.001f + 0.01f);
    }
  }
  ex += 0.5f;
  ey += 0.5f;
  uint32_t m = 0u;
  for (int w = 0; w < nwaves; ++w) {
    const Box b = wave_box(a, w, tx, ty);
    const bool hit = (u + ex >= b.x0) && (u - ex <= b.x1) && (v + ey >= b.y0) && (v - ey <= b.y1);
    m |= hit ? (1u << w) : 0u;
  }
  return m;
}

// Wave 0 turns the per-record wave masks of a batch into one ordered index
// list per wave (lane l handles batch entries 4l .. 4l+3).
__device__ __forceinline__ void build_wave_lists(const uint8_t* s_mask, int cnt, int nwaves, int stride,
                                                 uint8_t* s_list, int* s_len) {
  const int l = threadIdx.x;  // called by wave 0 only
  uint32_t m[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int i = 4 * l + q;
    m[q] = i < cnt ? s_mask[i] : 0u;
  }
  for (int w = 0; w < nwaves; ++w) {
    uint32_t c = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) c += (m[q] >> w) & 1u;
    uint32_t incl = c;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const uint32_t t = __shfl_up(incl, o, kWave);
      if (l >= o) incl += t;
    }
    uint32_t pos = incl - c;
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if ((m[q] >> w) & 1u) s_list[w * stride + pos++] = (uint8_t)(4 * l + q);
    if (l == kWave - 1) s_len[w] = (int)incl;
  }
}

// Dynamic LDS of the blend kernels, sized by the batch depth B and the wave count W:
//   records 3 x B float4 | [bwd] B pair indices | [bwd] W x B x 9 partial sums | B masks | 4 x B lists
struct Lds {
  float4 *a, *b, *c;
  uint32_t* e;
  float* part;
  uint8_t* mask;
  uint8_t* list;  // [4][B]
};

__host__ __device__ inline size_t lds_bytes(int batch, int nwaves, bool bwd) {
  size_t o = 3 * 16 * (size_t)batch;
  if (bwd) o += 4 * (size_t)batch + 4 * (size_t)GS_GRAD_FLOATS * nwaves * batch;
  o += (size_t)batch + 4 * (size_t)batch;
  return (o + 15) & ~(size_t)15;
}

__device__ inline Lds lds_carve(unsigned char* base, int batch, int nwaves, bool bwd) {
  Lds l;
  size_t o = 0;
  l.a = (float4*)(base + o), o += 16 * (size_t)batch;
  l.b = (float4*)(base + o), o += 16 * (size_t)batch;
  l.c = (float4*)(base + o), o += 16 * (size_t)batch;
  l.e = nullptr;
  l.part = nullptr;
  if (bwd) {
    l.e = (uint32_t*)(base + o), o += 4 * (size_t)batch;
    l.part = (float*)(base + o), o += 4 * (size_t)GS_GRAD_FLOATS * nwaves * batch;
  }
  l.mask = base + o, o += batch;
  l.list = base + o;
  return l;
}

// Largest backward batch: the partial sums of all waves stay within 18 KB.
__host__ __device__ inline int bwd_batch(int batch, int nwaves) {
  const int cap = 512 / nwaves;
  return batch < cap ? batch : cap;
}

template <int PPT, bool CULL>
__global__ __launch_bounds__(256) void render_fwd_kernel(RenderArgs a, ViewTable vt, float* __restrict__ image,
                                                         float* __restrict__ T_final, int32_t* __restrict__ last_out) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int s_len[4];
  __shared__ int s_alive[16];
  const int gtile = blockIdx.x;
  const TileCtx tc = tile_ctx(vt, a, gtile);
  const ViewArgs& va = vt.v[tc.view];
  const int nthreads = blockDim.x;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave, nwaves = nthreads / kWave;
  const Lds L = lds_carve(smem, a.batch, nwaves, false);
  float4* s_a = L.a;
  float4* s_b = L.b;
  float4* s_c = L.c;
  uint8_t* s_mask = L.mask;
  uint8_t* s_list = L.list;

  float px[PPT], py[PPT], T[PPT], C0[PPT], C1[PPT], C2[PPT];
  int last[PPT];
  bool done[PPT];
#pragma unroll
  for (int p = 0; p < PPT; ++p) {
    int x, y;
    pixel_of(a, PPT, threadIdx.x, p, tc.tx, tc.ty, &x, &y);
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
      const float4 ra = a.splats[(size_t)rec * 3 + 0];
      const float4 rb = a.splats[(size_t)rec * 3 + 1];
      s_a[i] = ra;
      s_b[i] = rb;
      s_c[i] = a.splats[(size_t)rec * 3 + 2];
      if (CULL) s_mask[i] = (uint8_t)footprint_mask(a, ra, rb, nwaves, tc.tx, tc.ty);
    }
    __syncthreads();
    int len = cnt;
    if (CULL) {
      if (wave == 0) build_wave_lists(s_mask, cnt, nwaves, a.batch, s_list, s_len);
      __syncthreads();
      len = s_len[wave];
    }
    for (int jj = 0; jj < len; ++jj) {
      const int j = CULL ? (int)s_list[wave * a.batch + jj] : jj;
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

template <int PPT, bool CULL>
__global__ __launch_bounds__(256) void render_bwd_kernel(RenderArgs a, ViewTable vt, const float* __restrict__ T_final,
                                                         const int32_t* __restrict__ last_in,
                                                         const float* __restrict__ dL_dimage,
                                                         float* __restrict__ grad_pair) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int s_len[4];
  __shared__ int s_max[16];
  const int gtile = blockIdx.x;
  const TileCtx tc = tile_ctx(vt, a, gtile);
  const ViewArgs& va = vt.v[tc.view];
  const int nthreads = blockDim.x;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave, nwaves = nthreads / kWave;
  const int64_t plane = (int64_t)va.W * va.H;
  const int batch = bwd_batch(a.batch, nwaves);
  const Lds L = lds_carve(smem, batch, nwaves, true);
  float4* s_a = L.a;
  float4* s_b = L.b;
  float4* s_c = L.c;
  uint32_t* s_e = L.e;
  float* s_part = L.part;  // per-wave partial sums of one batch: [nwaves][batch][9]
  uint8_t* s_mask = L.mask;
  uint8_t* s_list = L.list;

  float px[PPT], py[PPT], T[PPT], g0[PPT], g1[PPT], g2[PPT], RdL[PPT];
  int lc[PPT];
  int my_max = 0;
#pragma unroll
  for (int p = 0; p < PPT; ++p) {
    int x, y;
    pixel_of(a, PPT, threadIdx.x, p, tc.tx, tc.ty, &x, &y);
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

  // pairs behind every pixel's last contributor receive no gradient
  for (uint32_t i = tc.start + (uint32_t)maxlast + threadIdx.x; i < tc.end; i += nthreads) {
    float* gp = grad_pair + (size_t)a.pair_index[i] * GS_GRAD_FLOATS;
#pragma unroll
    for (int k = 0; k < GS_GRAD_FLOATS; ++k) gp[k] = 0.0f;
  }

  const uint32_t wend = tc.start + (uint32_t)maxlast;
  for (uint32_t be = wend; be > tc.start;) {
    const uint32_t bs = (be - tc.start > (uint32_t)batch) ? be - batch : tc.start;
    const int cnt = (int)(be - bs);
    for (int i = threadIdx.x; i < cnt; i += nthreads) {
      const uint32_t rec = a.ids[bs + i];
      const float4 ra = a.splats[(size_t)rec * 3 + 0];
      const float4 rb = a.splats[(size_t)rec * 3 + 1];
      s_e[i] = a.pair_index[bs + i];
      s_a[i] = ra;
      s_b[i] = rb;
      s_c[i] = a.splats[(size_t)rec * 3 + 2];
      if (CULL) s_mask[i] = (uint8_t)footprint_mask(a, ra, rb, nwaves, tc.tx, tc.ty);
    }
    for (int i = threadIdx.x; i < nwaves * batch * GS_GRAD_FLOATS; i += nthreads) s_part[i] = 0.0f;
    __syncthreads();
    int len = cnt;
    if (CULL) {
      if (wave == 0) build_wave_lists(s_mask, cnt, nwaves, batch, s_list, s_len);
      __syncthreads();
      len = s_len[wave];
    }
    for (int jj = len - 1; jj >= 0; --jj) {
      const int j = CULL ? (int)s_list[wave * batch + jj] : jj;
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
      if (__ballot(any) != 0) {  // wave-uniform
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
          float* part = &s_part[(wave * batch + j) * GS_GRAD_FLOATS];
          part[0] = gu;
          part[1] = gv;
          part[2] = gA;
          part[3] = gB;
          part[4] = gC;
          part[5] = go;
          part[6] = gr;
          part[7] = gg;
          part[8] = gb;
        }
      }
    }
    __syncthreads();
    // fixed-order sum over the waves, one store per (pair, attribute)
    for (int i = threadIdx.x; i < cnt * GS_GRAD_FLOATS; i += nthreads) {
      const int j = i / GS_GRAD_FLOATS, k = i - j * GS_GRAD_FLOATS;
      float v = s_part[j * GS_GRAD_FLOATS + k];
      for (int w = 1; w < nwaves; ++w) v += s_part[(w * batch + j) * GS_GRAD_FLOATS + k];
      grad_pair[(size_t)s_e[j] * GS_GRAD_FLOATS + k] = v;
    }
    __syncthreads();
    be = bs;
  }
}

static int tile_threads(const RenderArgs& a) { return (1 << (a.log2_tw + a.log2_th)) / a.ppt; }

template <int PPT>
static void fwd_ppt(const RenderArgs& a, const ViewTable& vt, float* image, float* T_final, int32_t* last,
                    hipStream_t s) {
  const int nt = tile_threads(a);
  const dim3 grid((unsigned)vt.total_tiles), block((unsigned)nt);
  const size_t sh = lds_bytes(a.batch, nt / kWave, false);
  if (a.cull)
    hipLaunchKernelGGL((render_fwd_kernel<PPT, true>), grid, block, sh, s, a, vt, image, T_final, last);
  else
    hipLaunchKernelGGL((render_fwd_kernel<PPT, false>), grid, block, sh, s, a, vt, image, T_final, last);
}

template <int PPT>
static void bwd_ppt(const RenderArgs& a, const ViewTable& vt, const float* T_final, const int32_t* last,
                    const float* dL, float* grad_pair, hipStream_t s) {
  const int nt = tile_threads(a);
  const dim3 grid((unsigned)vt.total_tiles), block((unsigned)nt);
  const size_t sh = lds_bytes(bwd_batch(a.batch, nt / kWave), nt / kWave, true);
  if (a.cull)
    hipLaunchKernelGGL((render_bwd_kernel<PPT, true>), grid, block, sh, s, a, vt, T_final, last, dL, grad_pair);
  else
    hipLaunchKernelGGL((render_bwd_kernel<PPT, false>), grid, block, sh, s, a, vt, T_final, last, dL, grad_pair);
}

hipError_t launch_render_fwd(const RenderArgs& a, const ViewTable& vt, float* image, float* T_final,
                             int32_t* last_contrib, hipStream_t s) {
  if (vt.total_tiles == 0) return hipSuccess;
  switch (a.ppt) {
    case 1: fwd_ppt<1>(a, vt, image, T_final, last_contrib, s); break;
    case 2: fwd_ppt<2>(a, vt, image, T_final, last_contrib, s); break;
    default: fwd_ppt<4>(a, vt, image, T_final, last_contrib, s); break;
  }
  return hipGetLastError();
}

hipError_t launch_render_bwd(const RenderArgs& a, const ViewTable& vt, const float* T_final,
                             const int32_t* last_contrib, const float* dL_dimage, float* grad_pair, hipStream_t s) {
  if (vt.total_tiles == 0) return hipSuccess;
  switch (a.ppt) {
    case 1: bwd_ppt<1>(a, vt, T_final, last_contrib, dL_dimage, grad_pair, s); break;
    case 2: bwd_ppt<2>(a, vt, T_final, last_contrib, dL_dimage, grad_pair, s); break;
    default: bwd_ppt<4>(a, vt, T_final, last_contrib, dL_dimage, grad_pair, s); break;
  }
  return hipGetLastError();
}

}  // namespace gs
