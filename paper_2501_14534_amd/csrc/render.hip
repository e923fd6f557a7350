// Per-tile front-to-back compositing (Eq. 2) and its backward.
//
// One workgroup per tile (global tile ids span all views of the call),
// launched in the heaviest-first order gs_bin_sort writes when the caller
// asks for it; each wave of it owns one sub-tile of pixels.  The backward
// walks the tile's sorted list in batches of splat records that the
// workgroup gathers into LDS together; the forward's waves walk the list
// independently (no workgroup barrier), each staging groups of 64 records
// into its own LDS with the gathers issued two groups ahead.  Every lane
// walks the staged records for its pixel(s), reading each as a wave-uniform
// LDS broadcast.  No MFMA: the work per (pixel, splat) pair is ~20 VALU
// operations and one exp.
//
// Sub-tile culling (CULL): while staging a batch, each record's conservative
// alpha >= 1/255 footprint (the ellipse q <= 2 ln(255 o'), widened by
// rounding margins) is tested against the live-pixel box of every wave: its
// bounding box first, then the ellipse itself (the minimum of q over the
// box); each wave then walks only the records whose bit it holds, taken from
// a ballot in scalar registers.  Culled records fail a per-pixel test for
// every pixel of that wave, so the result is unchanged.
//
// Forward: lanes whose pixels have terminated drop out of the walk through
// the exec mask, and a wave leaves once all its pixels are done; the
// backward's waves vote before each batch and the workgroup leaves once every
// pixel is done.  The forward evaluates four records' falloff and alpha
// together (independent of the transmittance) before compositing them in
// order.  Long lists can be split into forward chunks walked in parallel
// (a product pass gives each chunk its starting transmittance; see
// render_fwd_kernel), which shortens the critical path of the deepest tiles.
//
// Backward: the list is re-walked back to front from the tile's largest
// last_contrib; each pixel recovers the transmittance in front of a splat by
// dividing by (1 - alpha) and carries the dL/dC-weighted colour behind it, so
// no per-pixel list is stored.  Per-pair partials (9 floats) are summed over
// the lane's pixels, over the wave (a butterfly reduce-scatter over cross-lane
// swaps: about 30 instructions for all 9 sums), then over the workgroup's
// waves in a fixed order (LDS), and stored once per (tile, splat) at the
// pair's emission position: no atomics, so the result is bitwise reproducible.
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

// Box of pixel centres [x0, x1] x [y0, y1]; empty when x0 > x1.
struct Box {
  float x0, x1, y0, y1;
};

// Box of the pixel centres of this wave's lanes whose pixel is still live
// (may still composite or receive gradient), the same value in every lane.
// Culling against it instead of the wave's whole sub-tile drops the records
// that can only reach pixels that have already stopped.
// Min (or max) over the 64 lanes, returned in every lane: row shifts by 1, 2,
// 4, 8 leave each 16-lane row's result in its lane 15, row broadcasts 15 and
// 31 fold the rows into lane 63 (lanes without a source see the identity).
template <bool MAX>
__device__ __forceinline__ float wave_minmax(float v) {
  const int id = __builtin_bit_cast(int, MAX ? -__builtin_inff() : __builtin_inff());
  auto step = [&](float x, float y) { return MAX ? fmaxf(x, y) : fminf(x, y); };
#define GS_DPP_STEP(ctrl, rmask) \
  v = step(v, __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(id, __builtin_bit_cast(int, v), ctrl, rmask, 0xf, false)))
  GS_DPP_STEP(0x111, 0xf);
  GS_DPP_STEP(0x112, 0xf);
  GS_DPP_STEP(0x114, 0xf);
  GS_DPP_STEP(0x118, 0xf);
  GS_DPP_STEP(0x142, 0xa);
  GS_DPP_STEP(0x143, 0xc);
#undef GS_DPP_STEP
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), kWave - 1));
}

template <int PPT>
__device__ __forceinline__ Box live_box(const float (&px)[PPT], const float (&py)[PPT], const bool (&live)[PPT]) {
  Box b{__builtin_inff(), -__builtin_inff(), __builtin_inff(), -__builtin_inff()};
#pragma unroll
  for (int p = 0; p < PPT; ++p)
    if (live[p]) {
      b.x0 = fminf(b.x0, px[p]);
      b.x1 = fmaxf(b.x1, px[p]);
      b.y0 = fminf(b.y0, py[p]);
      b.y1 = fmaxf(b.y1, py[p]);
    }
  b.x0 = wave_minmax<false>(b.x0);
  b.x1 = wave_minmax<true>(b.x1);
  b.y0 = wave_minmax<false>(b.y0);
  b.y1 = wave_minmax<true>(b.y1);
  return b;
}

// Bit w set when record (u, v, conic, o', radius) may composite some pixel in
// wave w's live box.
// Minimum over the box dx in [X0, X1], dy in [Y0, Y1] (relative to the
// centre) of q = A dx^2 + 2 B dx dy + C dy^2, positive definite: 0 when the
// centre is inside, else on an edge, where the 1-D minimiser is clamped to
// the edge (iA = 1 / A, iC = 1 / C).
__device__ __forceinline__ float qmin_box(float A, float B, float C, float iA, float iC, float X0, float X1,
                                          float Y0, float Y1) {
  if (X0 <= 0.f && X1 >= 0.f && Y0 <= 0.f && Y1 >= 0.f) return 0.f;
  auto qv = [&](float dx, float dy) { return A * dx * dx + 2.0f * B * dx * dy + C * dy * dy; };
  const float dyx0 = fminf(fmaxf(-B * X0 * iC, Y0), Y1), dyx1 = fminf(fmaxf(-B * X1 * iC, Y0), Y1);
  const float dxy0 = fminf(fmaxf(-B * Y0 * iA, X0), X1), dxy1 = fminf(fmaxf(-B * Y1 * iA, X0), X1);
  return fminf(fminf(qv(X0, dyx0), qv(X1, dyx1)), fminf(qv(dxy0, Y0), qv(dxy1, Y1)));
}

__device__ __forceinline__ uint32_t footprint_mask(float4 ra, float4 rb, int nwaves, const Box* boxes) {
  const float u = ra.x, v = ra.y, A = ra.z, B = ra.w, C = rb.x, o = rb.y, r = rb.z;
  if (!(o >= kAlphaMin * 0.999f)) return 0u;  // alpha <= o' < 1/255 at every pixel
  float ex = r, ey = r, qm = 0.f, iA = 0.f, iC = 0.f;
  bool exact = false;
  const float det = A * C - B * B;
  if (det > 0.f) {
    const float tr = 0.5f * (A + C);
    const float lmax = tr + sqrtf(fmaxf(0.f, tr * tr - det));
    if (lmax * lmax <= 1e3f * det) {  // condition number <= 1e3: rounding of q stays far below the margins
      qm = 2.0f * __logf(255.0f * o) * 1.002f + 0.002f;
      const float idet = 1.0f / det;
      ex = fminf(r, sqrtf(fmaxf(qm, 0.f) * C * idet) * 1.001f + 0.01f);
      ey = fminf(r, sqrtf(fmaxf(qm, 0.f) * A * idet) * 1.001f + 0.01f);
      iA = 1.0f / A;
      iC = 1.0f / C;
      exact = true;
    }
  }
  ex += 0.5f;
  ey += 0.5f;
  uint32_t m = 0u;
  for (int w = 0; w < nwaves; ++w) {
    const Box b = boxes[w];
    bool hit = (u + ex >= b.x0) && (u - ex <= b.x1) && (v + ey >= b.y0) && (v - ey <= b.y1);
    // the ellipse q <= qm against the box of pixel centres (widened by 1e-3 px):
    // its bounding box can reach a corner of the box that the ellipse misses
    if (hit && exact)
      hit = qmin_box(A, B, C, iA, iC, b.x0 - 1e-3f - u, b.x1 + 1e-3f - u, b.y0 - 1e-3f - v, b.y1 + 1e-3f - v) <= qm;
    m |= hit ? (1u << w) : 0u;
  }
  return m;
}

// Entry selection.  Once a batch is staged, lane l of wave w reads the
// footprint mask of entry 64c + l; the ballot is the set of entries of chunk c
// that wave w walks.  The walk takes the set bits in order from scalar
// registers, so no per-wave index list is built, stored or read.
template <bool CULL>
__device__ __forceinline__ uint64_t chunk_bits(const uint8_t* s_mask, int c, int cnt, int wave, int lane) {
  const int i = c * kWave + lane;
  bool bit = i < cnt;
  if (CULL && bit) bit = ((s_mask[i] >> wave) & 1u) != 0u;
  return __ballot(bit);
}

// Dynamic LDS of the blend kernels, sized by the batch depth B and the wave count W:
//   records 3 x B float4 | [bwd] B pair indices | [bwd] W x B x 9 partial sums | B masks
struct Lds {
  float4 *a, *b, *c;
  uint32_t* e;
  float* part;
  uint8_t* mask;
};

__host__ __device__ inline size_t lds_bytes(int batch, int nwaves, bool bwd) {
  size_t o = 3 * 16 * (size_t)batch;
  if (bwd) o += 4 * (size_t)batch + 4 * (size_t)GS_GRAD_FLOATS * nwaves * batch;
  o += (size_t)batch;
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
  l.mask = base + o;
  return l;
}

// Largest backward batch: the partial sums of all waves stay within 18 KB.
__host__ __device__ inline int bwd_batch(int batch, int nwaves) {
  const int cap = 512 / nwaves;
  return batch < cap ? batch : cap;
}

__device__ __forceinline__ int tile_of_block(const RenderArgs& a) {
  return a.order ? (int)a.order[blockIdx.x] : (int)blockIdx.x;
}

// Cross-lane moves of the backward's reduce-scatter.  permlane32_swap
// exchanges the upper 32 lanes of its first operand with the lower 32 lanes
// of its second, permlane16_swap the odd 16-lane rows of the first with the
// even rows of the second (both new on gfx950).  The pair result is read
// through a 64-bit cast.
__device__ __forceinline__ void swap_halves(float& a, float& b) {
  const uint64_t r = __builtin_bit_cast(
      uint64_t, __builtin_amdgcn_permlane32_swap(__builtin_bit_cast(uint32_t, a), __builtin_bit_cast(uint32_t, b),
                                                 false, false));
  a = __builtin_bit_cast(float, (uint32_t)r);
  b = __builtin_bit_cast(float, (uint32_t)(r >> 32));
}

__device__ __forceinline__ void swap_rows(float& a, float& b) {
  const uint64_t r = __builtin_bit_cast(
      uint64_t, __builtin_amdgcn_permlane16_swap(__builtin_bit_cast(uint32_t, a), __builtin_bit_cast(uint32_t, b),
                                                 false, false));
  a = __builtin_bit_cast(float, (uint32_t)r);
  b = __builtin_bit_cast(float, (uint32_t)(r >> 32));
}

template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xf, 0xf, false));
}

// Sums each of the 9 per-lane values over the 64 lanes of the wave
// (butterfly reduce-scatter: every step halves the values a lane carries).
// Element e ends in the four lanes l with (l >> 2) bits giving
// k2 = 2 b3 + b2 <= 2, k1 = k2 + 3 b4 <= 4, e = k1 + 5 b5 <= 8; the tree is
// fixed, so the sum is reproducible.  Needs every lane of the wave active.
__device__ __forceinline__ float reduce_scatter9(const float (&x)[GS_GRAD_FLOATS], bool b2, bool b3) {
  float y[5];  // lane bit 5: elements 0-4 stay in lanes 0-31, 5-8 go to lanes 32-63
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    float lo = x[k], hi = k + 5 < GS_GRAD_FLOATS ? x[k + 5] : 0.0f;
    swap_halves(lo, hi);
    y[k] = lo + hi;
  }
  float z[3];  // lane bit 4: y0-y2 stay in even rows, y3-y4 go to odd rows
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    float lo = y[k], hi = k + 3 < 5 ? y[k + 3] : 0.0f;
    swap_rows(lo, hi);
    z[k] = lo + hi;
  }
  // lane bit 3: row_mirror pairs lane i of a row with lane 15 - i
  const float t0 = z[0] + dpp_f<0x140>(z[0]);
  const float t1 = z[1] + dpp_f<0x140>(z[1]);
  const float t2 = z[2] + dpp_f<0x140>(z[2]);
  const float w0 = b3 ? t2 : t0;
  const float w1 = b3 ? 0.0f : t1;
  // lane bit 2: row_half_mirror pairs lane i of an 8-lane half row with lane 7 - i
  const float u0 = w0 + dpp_f<0x141>(w0);
  const float u1 = w1 + dpp_f<0x141>(w1);
  float v = b2 ? u1 : u0;
  // lane bits 1 and 0: quad permutations [2,3,0,1] and [1,0,3,2]
  v += dpp_f<0x4E>(v);
  v += dpp_f<0xB1>(v);
  return v;
}

// Walk modes of the forward kernel.
//   kFull:  Eq. 2 over one forward chunk of a tile's list (the whole list when
//           forward chunking is off): the image, or the chunk's results.
//   kCount: the same walk, counting instead of blending: per Gaussian, the
//           number of pixels where it is composited (the ray hits of Eq. 4),
//           added to a.hits; no image, no chunk states.  Per record and batch,
//           the waves add their ballot counts into an LDS counter (in place
//           of the staged colours), flushed to the Gaussian's global counter
//           once the batch is walked.
//   kTPass: the product of (1 - alpha) over the chunk's splats that pass the
//           skip and square tests, ignoring the stop rule (stopped once under
//           1e-4, where its value no longer matters).
//
// Forward chunking.  A list longer than F = 2^log2_fchunk entries is split
// into chunks [start + kF, start + (k+1)F).  Three launches: every tile's
// first chunk (the only launch without chunking), which also leaves each
// pixel's transmittance after it (0 if it stopped) as the product P_0; the
// product pass over chunks 1 .. m-2, for the pixels still going after chunk
// 0 only; the full walk of chunks 1 .. m-1.  Chunk k starts from T_in =
// P_0 ... P_{k-1}: a pixel whose product fell under 1e-4 stopped in an
// earlier chunk (T only decreases), and otherwise T_in is its transmittance.
// Each chunk of a long list stores its colour, final T and last index;
// fwd_combine_kernel adds them up.  The critical path of a deep tile becomes
// about three chunks instead of its whole list.
enum : int { kFull = 0, kCount = 1, kTPass = 2 };
constexpr int kHalves = 2;  // entries a lane stages per forward group
// records evaluated together by the forward walk: four independent chains a
// lane (PPT pixels per record)
template <int PPT>
constexpr int ilp_records() { return PPT >= 4 ? 1 : 4 / PPT; }

// Stores and loads of the values one work item hands to another within a
// launch (image, T_final, last_contrib, chunk states).  COH: agent-scope
// relaxed atomics, which go to the device's coherence point instead of a
// compute die's L2, so an item on another die sees them once the flag that
// follows them is seen, without a cache-wide writeback or invalidate.
template <bool COH, typename T>
__device__ __forceinline__ void put(T* p, T v) {
  if (COH)
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else
    *p = v;
}
template <bool COH>
__device__ __forceinline__ void put4(float4* p, float4 v) {
  float* f = (float*)p;
  put<COH>(f + 0, v.x);
  put<COH>(f + 1, v.y);
  put<COH>(f + 2, v.z);
  put<COH>(f + 3, v.w);
}
template <bool COH, typename T>
__device__ __forceinline__ T get(const T* p) {
  return COH ? __hip_atomic_load(const_cast<T*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : *p;
}
template <bool COH>
__device__ __forceinline__ float4 get4(const float4* p) {
  const float* f = (const float*)p;
  return make_float4(get<COH>(f + 0), get<COH>(f + 1), get<COH>(f + 2), get<COH>(f + 3));
}

// One work item of a forward walk.  s_rec / s_cnt: per wave, the staged group
// of records (a, b, c) and (COUNT) its hit counts.  Items [0, nfslots) are
// the forward chunks that start at a forward boundary (slot order); the rest
// are each tile's first chunk, in the tile schedule.  Counting walks have no
// chunk items.  Returns the largest last_contrib this thread stored (0 if none).
template <int PPT, bool CULL, int MODE, bool COH = false>
__device__ __forceinline__ int fwd_item(const RenderArgs& a, const ViewTable& vt, float* __restrict__ image,
                                         float* __restrict__ T_final, int32_t* __restrict__ last_out, int64_t item,
                                         float4 (*s_rec)[3][kHalves * kWave], uint32_t (*s_cnt)[kHalves * kWave]) {
  constexpr bool COUNT = MODE == kCount, TPASS = MODE == kTPass;
  const int lf = COUNT ? 31 : a.log2_fchunk;
  const int64_t nfs = COUNT ? 0 : a.nfslots;
  int gtile;
  bool first;
  if (item < nfs) {
    const uint32_t owner = a.fslot_owner[item];
    if (owner >= (uint32_t)vt.total_tiles) return 0;  // no boundary here (uniform)
    gtile = (int)owner;
    first = false;
  } else {
    const int b = (int)(item - nfs);
    gtile = a.order ? (int)a.order[b] : b;
    first = true;
  }
  const TileCtx tc = tile_ctx(vt, a, gtile);
  const uint64_t fmask = (1ull << lf) - 1;
  const uint64_t cs64 = first ? (uint64_t)tc.start : (((uint64_t)item << lf) | ((uint64_t)tc.start & fmask));
  if (!first && !(cs64 > (uint64_t)tc.start && cs64 < (uint64_t)tc.end)) return 0;  // a record not of this list
  const uint32_t cs = (uint32_t)cs64;
  const uint32_t ce = (uint32_t)min(cs64 + (1ull << lf), (uint64_t)tc.end);
  const uint32_t len = tc.end - tc.start;
  const uint32_t nfc = len == 0 ? 1u : (uint32_t)(((uint64_t)len + fmask) >> lf);  // forward chunks of the list
  const uint32_t kf = (uint32_t)((cs64 - tc.start) >> lf);                           // this chunk
  if (TPASS && (kf == 0 || kf + 1 == nfc)) return 0;  // chunk 0 leaves its own; the last one is not needed
  const ViewArgs& va = vt.v[tc.view];
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  float4* s_a = s_rec[wave][0];
  float4* s_b = s_rec[wave][1];
  float4* s_c = s_rec[wave][2];
  uint32_t* s_hits = s_cnt[wave];  // COUNT only
  if (COUNT) {
#pragma unroll
    for (int h = 0; h < kHalves; ++h) s_hits[h * kWave + lane] = 0u;
  }

  // C: colour composited so far (the image, summed in list order whatever
  // the tiling); S: colour composited since the last chunk boundary (kept
  // apart so that the colour after a boundary is a sum of non-negative
  // segments, accurate relative to itself)
  float px[PPT], py[PPT], T[PPT], C0[PPT], C1[PPT], C2[PPT], S0[PPT], S1[PPT], S2[PPT];
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
    S0[p] = S1[p] = S2[p] = 0.0f;
    last[p] = 0;
    done[p] = !(x < va.W && y < va.H);
  }

  const int tpx = 1 << (a.log2_tw + a.log2_th);
  const int lc = (COUNT || TPASS) ? 31 : a.log2_chunk;  // counting and products record no chunk states
  // chunk k >= 1 starts from the product of the earlier chunks' products
  bool dead[PPT];
#pragma unroll
  for (int p = 0; p < PPT; ++p) dead[p] = false;
  if (MODE == kFull && kf > 0) {
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
      float t = 1.0f;
      for (uint32_t j = 1; j <= kf; ++j)
        t *= a.fprod[(int64_t)(((uint64_t)tc.start + ((uint64_t)j << lf)) >> lf) * tpx + threadIdx.x * PPT + p];
      T[p] = t;
      dead[p] = !done[p] && t < kTMin;
      done[p] = done[p] || dead[p];
    }
  }
  if (TPASS) {  // only the pixels still going after chunk 0
    const float* p0 = a.fprod + (int64_t)(((uint64_t)tc.start + (1ull << lf)) >> lf) * tpx;
#pragma unroll
    for (int p = 0; p < PPT; ++p) done[p] = done[p] || p0[threadIdx.x * PPT + p] < kTMin;
  }
  int nbnd = 0;  // chunk boundaries this wave recorded (uniform in the wave)
  // first backward boundary this walk can record: the first multiple of 2^lc
  // (relative to the list start) at or after cs, never the list start
  uint64_t b0 = (uint64_t)tc.start + ((((uint64_t)cs - tc.start) + ((1ull << lc) - 1)) >> lc << lc);
  if (b0 == (uint64_t)tc.start) b0 += 1ull << lc;
  // Each wave walks its own sub-tile independently (no workgroup barrier), in
  // groups of up to kHalves x 64 entries (batch_depth if smaller) that never
  // straddle a chunk boundary: lane l stages entries l and 64 + l of the group
  // into the wave's LDS, with their culling bits for the wave's live box.  The
  // records of group g + 1 are loaded into the registers group g was just
  // staged from, while group g is walked, and the ids of group g + 2 with them.
  // Late in a deep list most records are culled and a group's walk is much
  // shorter than a gather's latency, so a walk that lone waves take (the
  // deepest lists) is bound by one latency per group: two entries a lane halve
  // the groups.  (Deeper prefetching across groups is undone by the waits the
  // compiler puts in front of loop-carried loads.)
  constexpr uint32_t GH = kWave;                         // entries per half group
  const uint32_t G = (uint32_t)min(kHalves * kWave, a.batch);
  auto group_end = [&](uint32_t b) -> uint32_t {
    const uint64_t rel = b - tc.start;
    const uint64_t next = (uint64_t)tc.start + (((rel >> lc) + 1) << lc);
    return (uint32_t)min(min((uint64_t)ce, (uint64_t)b + G), next);
  };
  uint32_t gs = cs;                                // group g: [gs, ge)
  uint32_t ge = gs < ce ? group_end(gs) : gs;      // g + 1: [ge, ge2)
  uint32_t ge2 = ge < ce ? group_end(ge) : ge;     // g + 2: [ge2, ge3)
  const float4 zf4 = make_float4(0.f, 0.f, 0.f, 0.f);
  float4 ra[kHalves], rb[kHalves], rc[kHalves];  // records of entries l, 64 + l of the group staged next
  uint32_t rid[kHalves], nid[kHalves];           // their ids; the ids of the group after it
  // every lane loads: a lane past a group's end takes the list's last entry,
  // which is never staged (a load under a lane condition leaves a merged value
  // whose register copy waits for the load)
  const uint32_t elast = tc.end - 1;  // used only when the walk has entries
#pragma unroll
  for (int h = 0; h < kHalves; ++h) {
    ra[h] = rb[h] = rc[h] = zf4;
    rid[h] = nid[h] = 0;
  }
  if (cs < ce) {
#pragma unroll
    for (int h = 0; h < kHalves; ++h) {
      rid[h] = a.ids[min(gs + h * GH + lane, elast)];
      nid[h] = a.ids[min(ge + h * GH + lane, elast)];
    }
#pragma unroll
    for (int h = 0; h < kHalves; ++h) {
      ra[h] = a.splats[(size_t)rid[h] * 3 + 0];
      rb[h] = a.splats[(size_t)rid[h] * 3 + 1];
      if (!COUNT) rc[h] = a.splats[(size_t)rid[h] * 3 + 2];
    }
  }
  while (gs < ce) {
    bool alive = false, live[PPT];
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
      live[p] = !done[p];
      alive |= live[p];
    }
    if (__ballot(alive) == 0) break;  // every pixel of this wave has stopped
    const uint64_t rel = gs - tc.start;
    if (MODE == kFull && rel != 0 && (rel & ((1ull << lc) - 1)) == 0) {
      // a chunk boundary of the backward: record each pixel's transmittance
      // here and the colour of the chunk that ends here, then start a new chunk
      const int64_t slot = (int64_t)(gs >> lc);
      float4* st = a.state + slot * tpx;
#pragma unroll
      for (int p = 0; p < PPT; ++p) {
        put4<COH>(st + threadIdx.x * PPT + p, make_float4(T[p], S0[p], S1[p], S2[p]));
        S0[p] = S1[p] = S2[p] = 0.0f;
      }
      if (lane == 0) a.slot_owner[slot] = (uint32_t)gtile;  // every wave that gets here writes the same
      ++nbnd;
    }
    const int cnt = (int)(ge - gs);
    Box box;
    if (CULL) box = live_box<PPT>(px, py, live);  // all lanes: a cross-lane reduction
    bool bits[kHalves];
    uint32_t gid[kHalves];
#pragma unroll
    for (int h = 0; h < kHalves; ++h) {
      const int e = h * (int)GH + lane;
      bits[h] = e < cnt;
      if (bits[h]) {  // entry e from the registers
        s_a[e] = staged_a(ra[h]);
        s_b[e] = staged_b(rb[h]);
        if (!COUNT) s_c[e] = rc[h];
        if (CULL) bits[h] = footprint_mask(ra[h], rb[h], 1, &box) != 0u;
      }
      gid[h] = rid[h];
    }
    // group g + 1's record loads into the registers just staged from, and
    // group g + 2's id loads
    const uint32_t ge3 = ge2 < ce ? group_end(ge2) : ge2;
#pragma unroll
    for (int h = 0; h < kHalves; ++h) {
      rid[h] = nid[h];
      ra[h] = a.splats[(size_t)rid[h] * 3 + 0];
      rb[h] = a.splats[(size_t)rid[h] * 3 + 1];
      if (!COUNT) rc[h] = a.splats[(size_t)rid[h] * 3 + 2];
    }
    if (ge < ce) {  // uniform; elast is an entry of the walk here
#pragma unroll
      for (int h = 0; h < kHalves; ++h) nid[h] = a.ids[min(ge2 + h * GH + lane, elast)];
    }
    wave_lds_sync();  // the staged group is visible to the whole wave
#pragma unroll
    for (int h = 0; h < kHalves; ++h) {
    uint64_t m = __ballot(bits[h]);
    if (m != 0) {
      // composite one evaluated record into this lane's pixel(s); branch-free: a
      // lane that skips the splat adds exact zeros
      auto composite = [&](int j, const Eval (&e)[PPT], const bool (&inside)[PPT], const float4& rc) {
        const int idx = (int)(gs + j - tc.start) + 1;
        uint32_t taken = 0;  // COUNT: pixels of this wave that composite record j
#pragma unroll
        for (int p = 0; p < PPT; ++p) {
          const bool use = !done[p] && inside[p] && !(e[p].alpha < kAlphaMin);
          const float Tn = T[p] * (1.0f - e[p].alpha);
          const bool stop = use && Tn < kTMin;  // stop before this splat
          done[p] = done[p] || stop;
          // the product pass multiplies the stopping splat in as well
          const bool take = TPASS ? use : use && !stop;
          const float w = take ? e[p].alpha * T[p] : 0.0f;
          C0[p] += rc.x * w;
          C1[p] += rc.y * w;
          C2[p] += rc.z * w;
          S0[p] += rc.x * w;
          S1[p] += rc.y * w;
          S2[p] += rc.z * w;
          T[p] = take ? Tn : T[p];
          last[p] = take ? idx : last[p];
          if (COUNT) taken += (uint32_t)__popcll(__ballot(take));
        }
        if (COUNT && lane == 0 && taken != 0) s_hits[j] += taken;
      };
      // R records at a time (in list order) while R are left: their falloff
      // and alpha do not depend on the transmittance, so the R evaluations run
      // as independent chains before the R dependent compositing steps (no
      // record is guarded on its own, which would let the compiler sink each
      // evaluation next to its compositing step and serialise the
      // exponentials' latencies); the last ones one at a time.
      const float4 zero4 = make_float4(0.f, 0.f, 0.f, 0.f);
      auto eval_one = [&](int j, Eval (&e)[PPT], bool (&in)[PPT], float4& rc) {
        const float4 ra = s_a[j], rb = s_b[j];
        rc = COUNT ? zero4 : s_c[j];
#pragma unroll
        for (int p = 0; p < PPT; ++p)
          in[p] = eval_splat_all(px[p], py[p], ra.x, ra.y, ra.z, ra.w, rb.x, rb.y, rb.z, &e[p]);
      };
      constexpr int R = ilp_records<PPT>();
      const int hoff = h * (int)GH;  // bit b of m is entry hoff + b
      while (m != 0) {
        if (R == 1 || __popcll(m) >= R) {  // wave-uniform
          int jq[R];
#pragma unroll
          for (int q = 0; q < R; ++q) {
            jq[q] = hoff + __builtin_ctzll(m);
            m &= m - 1;
          }
          float4 rcq[R];
          Eval eq[R][PPT];
          bool iq[R][PPT];
#pragma unroll
          for (int q = 0; q < R; ++q) eval_one(jq[q], eq[q], iq[q], rcq[q]);
#pragma unroll
          for (int q = 0; q < R; ++q) composite(jq[q], eq[q], iq[q], rcq[q]);
        } else {
          const int j = hoff + __builtin_ctzll(m);
          m &= m - 1;
          float4 rc;
          Eval e[PPT];
          bool in[PPT];
          eval_one(j, e, in, rc);
          composite(j, e, in, rc);
        }
      }
      if (COUNT) {
        // flush the half's counters: lane l adds entry hoff + l's hits to its Gaussian
        wave_lds_sync();
        const uint32_t hv = hoff + lane < cnt ? s_hits[hoff + lane] : 0u;
        if (hv != 0) {
          atomicAdd(a.hits + ((int64_t)gid[h] - (int64_t)tc.view * a.n), hv);
          s_hits[hoff + lane] = 0u;
        }
      }
    }
    }
    wave_lds_sync();  // every lane has read the group before the next one overwrites it
    gs = ge;
    ge = ge2;
    ge2 = ge3;
  }

  if (COUNT) return 0;
  if (TPASS) {  // the product, at the boundary that ends this chunk
    float* fp = a.fprod + (int64_t)((uint64_t)ce >> lf) * tpx;
#pragma unroll
    for (int p = 0; p < PPT; ++p) fp[threadIdx.x * PPT + p] = T[p];
    return 0;
  }
  // Each recorded state becomes (T there, colour composited after it within
  // this walk): the suffix sums of the segments' colours, last one first.  The
  // states are read kSuf at a time, all loads in flight together (a deep list
  // records dozens of states, and one load at a time would put as many memory
  // round trips on the walk's critical path).
  constexpr int kSuf = PPT >= 4 ? 1 : 4 / PPT;
  for (int k0 = nbnd - 1; k0 >= 0; k0 -= kSuf) {
    float4 v[kSuf][PPT];
#pragma unroll
    for (int i = 0; i < kSuf; ++i) {
      if (k0 - i < 0) break;  // wave-uniform
      const int64_t slot = (int64_t)((b0 + ((uint64_t)(k0 - i) << lc)) >> lc);
#pragma unroll
      for (int p = 0; p < PPT; ++p) v[i][p] = get4<COH>(a.state + slot * tpx + threadIdx.x * PPT + p);
    }
#pragma unroll
    for (int i = 0; i < kSuf; ++i) {
      if (k0 - i < 0) break;
      const int64_t slot = (int64_t)((b0 + ((uint64_t)(k0 - i) << lc)) >> lc);
#pragma unroll
      for (int p = 0; p < PPT; ++p) {
        const float e0 = v[i][p].y, e1 = v[i][p].z, e2 = v[i][p].w;  // colour of the chunk before the boundary
        put4<COH>(a.state + slot * tpx + threadIdx.x * PPT + p, make_float4(v[i][p].x, S0[p], S1[p], S2[p]));
        S0[p] = e0 + S0[p];
        S1[p] = e1 + S1[p];
        S2[p] = e2 + S2[p];
      }
    }
  }

  if (nfc > 1) {
    // one chunk of several: its colour, final T and last index (-1: the pixel
    // had stopped before the chunk), at the boundary that ends it, or for the
    // last chunk at the one that starts it (second half of the arrays); the
    // first chunk also leaves P_0 (0 for the pixels that stopped in it)
    const int64_t idx = kf + 1 < nfc ? (int64_t)((uint64_t)ce >> lf) : a.nfslots + (int64_t)((uint64_t)cs >> lf);
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
      a.fres[idx * tpx + threadIdx.x * PPT + p] = make_float4(C0[p], C1[p], C2[p], T[p]);
      a.flast[idx * tpx + threadIdx.x * PPT + p] = dead[p] ? -1 : last[p];
      if (kf == 0) a.fprod[idx * tpx + threadIdx.x * PPT + p] = done[p] ? 0.0f : T[p];
    }
    return 0;
  }
  const int64_t plane = (int64_t)va.W * va.H;
  int my_max = 0;
#pragma unroll
  for (int p = 0; p < PPT; ++p) {
    const int x = (int)px[p], y = (int)py[p];
    if (x < va.W && y < va.H) {
      const int64_t pix = (int64_t)y * va.W + x;
      float* img = image + 3 * (int64_t)va.pix_off;
      put<COH>(img + pix, C0[p] + T[p] * a.bg[0]);
      put<COH>(img + plane + pix, C1[p] + T[p] * a.bg[1]);
      put<COH>(img + 2 * plane + pix, C2[p] + T[p] * a.bg[2]);
      put<COH>(T_final + va.pix_off + pix, T[p]);
      put<COH>(last_out + va.pix_off + pix, last[p]);
      my_max = max(my_max, last[p]);
    }
  }
  return my_max;
}

// Work items [item_base, item_base + gridDim.x) of a forward walk, one per workgroup.
// At one pixel a thread the kernel is held to 80 registers (six waves per SIMD).
template <int PPT, bool CULL, int MODE>
__global__ __launch_bounds__(256, PPT == 1 ? 6 : 1) void render_fwd_kernel(RenderArgs a, ViewTable vt,
                                                                           float* __restrict__ image,
                                                                           float* __restrict__ T_final,
                                                                           int32_t* __restrict__ last_out,
                                                                           int64_t item_base) {
  __shared__ float4 s_rec[4][3][kHalves * kWave];
  __shared__ uint32_t s_cnt[4][kHalves * kWave];
  fwd_item<PPT, CULL, MODE>(a, vt, image, T_final, last_out, (int64_t)blockIdx.x + item_base, s_rec, s_cnt);
}

// Forward chunking: the tiles with several chunks.  Per pixel, the chunks'
// colours are added from the last one down (giving the colour composited
// from each forward boundary on, which the backward adds to its chunk
// states), the final T is the one of the last chunk the pixel entered alive,
// and the last index the largest.  One workgroup per tile, in the schedule.
template <int PPT>
__global__ __launch_bounds__(256) void fwd_combine_kernel(RenderArgs a, ViewTable vt, float* __restrict__ image,
                                                          float* __restrict__ T_final,
                                                          int32_t* __restrict__ last_out) {
  const int gtile = tile_of_block(a);
  const TileCtx tc = tile_ctx(vt, a, gtile);
  const int lf = a.log2_fchunk;
  const uint32_t len = tc.end - tc.start;
  const uint32_t nfc = (uint32_t)(((uint64_t)len + ((1ull << lf) - 1)) >> lf);
  if (nfc < 2) return;
  const ViewArgs& va = vt.v[tc.view];
  const int tpx = 1 << (a.log2_tw + a.log2_th);
  const int64_t plane = (int64_t)va.W * va.H;
#pragma unroll
  for (int p = 0; p < PPT; ++p) {
    int x, y;
    pixel_of(a, PPT, threadIdx.x, p, tc.tx, tc.ty, &x, &y);
    const int q = threadIdx.x * PPT + p;
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, Tf = 1.f;
    bool have_T = false;
    int last = 0;
    for (int k = (int)nfc - 1; k >= 0; --k) {
      const uint64_t bk = (uint64_t)tc.start + ((uint64_t)k << lf);
      const int64_t idx = k + 1 < (int)nfc ? (int64_t)((bk + (1ull << lf)) >> lf) : a.nfslots + (int64_t)(bk >> lf);
      const float4 r = a.fres[idx * tpx + q];
      const int l = a.flast[idx * tpx + q];
      s0 = r.x + s0;
      s1 = r.y + s1;
      s2 = r.z + s2;
      if (k > 0) a.fsuf[(int64_t)(bk >> lf) * tpx + q] = make_float4(s0, s1, s2, 0.f);
      if (!have_T && l >= 0) {
        Tf = r.w;
        have_T = true;
      }
      last = max(last, l);
    }
    if (x < va.W && y < va.H) {
      const int64_t pix = (int64_t)y * va.W + x;
      float* img = image + 3 * (int64_t)va.pix_off;
      img[pix] = s0 + Tf * a.bg[0];
      img[plane + pix] = s1 + Tf * a.bg[1];
      img[2 * plane + pix] = s2 + Tf * a.bg[2];
      T_final[va.pix_off + pix] = Tf;
      last_out[va.pix_off + pix] = last;
    }
  }
}

// Owners of the forward boundaries: slot (start + kF) >> log2_fchunk of a
// tile's list, k >= 1.  One thread per tile.
__global__ void fwd_mark_kernel(RenderArgs a, int total_tiles) {
  const int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gt >= total_tiles || *a.status != 0) return;
  const uint64_t start = a.ranges[2 * gt], end = a.ranges[2 * gt + 1];
  const int lf = a.log2_fchunk;
  for (uint64_t q = start + (1ull << lf); q < end; q += 1ull << lf) a.fslot_owner[q >> lf] = (uint32_t)gt;
}

constexpr float kPosScale = 2.77258872223978124f;  // 4 ln 2 = -2 / kQScale

// The loss gradient a backward walk reads: dL/dimage from memory, or (fused
// with the forward) the mean-squared-error gradient computed per pixel from
// the image the forward wrote and the target, dL = scale_v (image - target)
// in single precision, as gs_l2_grad computes it; the tile's first backward
// item also stores it when dL_out is given.
struct LossIn {
  const float* dL_dimage;
  const float* image;
  const float* target;
  float* dL_out;
  float scale[GS_MAX_VIEWS];
};

// One work item of the backward walk.  Items [0, nslots) are the chunks that
// start at a recorded boundary (slot order, so the long lists' chunks start
// first); the rest are each tile's first chunk, in the tile schedule.  smem:
// lds_bytes(bwd_batch(batch, waves), waves, true) bytes.  ok false (a wait for
// the tile's forward that timed out): the item's loss gradient is NaN.  walked
// >= 0: the tile's largest last_contrib, known beforehand.
template <int PPT, bool CULL, bool L2>
__device__ __forceinline__ void bwd_item(const RenderArgs& a, const ViewTable& vt, const float* __restrict__ T_final,
                                         const int32_t* __restrict__ last_in, const LossIn& loss,
                                         float* __restrict__ grad_pair, int64_t item, unsigned char* smem,
                                         bool ok = true, int walked = -1) {
  __shared__ int s_max[4];
  __shared__ Box s_box[4];
  const int lg = a.log2_chunk;
  int gtile;
  bool first;
  if (item < a.nslots) {
    const uint32_t owner = a.slot_owner[item];
    if (owner >= (uint32_t)vt.total_tiles) return;  // no boundary here (uniform)
    gtile = (int)owner;
    first = false;
  } else {
    const int b = (int)(item - a.nslots);
    gtile = a.order ? (int)a.order[b] : b;
    first = true;
  }
  const TileCtx tc = tile_ctx(vt, a, gtile);
  const uint64_t cmask = (1ull << lg) - 1;
  // chunk [cs, ce) of the tile's list [start, end)
  const uint64_t cs = first ? (uint64_t)tc.start : (((uint64_t)item << lg) | ((uint64_t)tc.start & cmask));
  const uint64_t ce = min(cs + (1ull << lg), (uint64_t)tc.end);
  if (!first && !(cs > (uint64_t)tc.start && cs < (uint64_t)tc.end)) return;  // a record not of this list
  // a chunk at or past the tile's largest last_contrib has nothing to do (uniform)
  if (!first && walked >= 0 && cs >= (uint64_t)tc.start + (uint64_t)walked) return;
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

  // this lane's element of the reduce-scatter (see reduce_scatter9)
  const bool b2 = (lane >> 2) & 1, b3 = (lane >> 3) & 1;
  const int k2 = 2 * (int)b3 + (int)b2, k1 = k2 + 3 * ((lane >> 4) & 1), my_e = k1 + 5 * ((lane >> 5) & 1);
  const bool writer = (lane & 3) == 0 && k2 <= 2 && k1 <= 4 && my_e < GS_GRAD_FLOATS;
  // per element, the factor the walk leaves out: with m = -2 dL/dq,
  // dL/d(u, v) = (-2/k) dL/dq (A dx + B dy, B dx + C dy) = -(2 ln 2) m (a dx + b/2 dy, ...),
  // dL/d(A, B, C) = dL/dq (dx^2, 2 dx dy, dy^2) = -m (dx^2 / 2, dx dy, dy^2 / 2)
  const float escale = my_e < 2 ? -0.5f * kPosScale : my_e == 3 ? -1.0f : my_e < 5 ? -0.5f : 1.0f;

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
      const int64_t e0 = 3 * (int64_t)va.pix_off + pix;
      T[p] = get<L2>(T_final + va.pix_off + pix);
      lc[p] = get<L2>(last_in + va.pix_off + pix);
      if (L2) {
        const float sc = ok ? loss.scale[tc.view] : __builtin_nanf("");
        g0[p] = sc * (get<L2>(loss.image + e0) - loss.target[e0]);
        g1[p] = sc * (get<L2>(loss.image + e0 + plane) - loss.target[e0 + plane]);
        g2[p] = sc * (get<L2>(loss.image + e0 + 2 * plane) - loss.target[e0 + 2 * plane]);
        if (first && loss.dL_out) {
          loss.dL_out[e0] = g0[p];
          loss.dL_out[e0 + plane] = g1[p];
          loss.dL_out[e0 + 2 * plane] = g2[p];
        }
      } else {
        g0[p] = loss.dL_dimage[e0];
        g1[p] = loss.dL_dimage[e0 + plane];
        g2[p] = loss.dL_dimage[e0 + 2 * plane];
      }
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
  const uint64_t wlim = (uint64_t)tc.start + (uint64_t)maxlast;

  // Pairs behind every pixel's last contributor receive no gradient: their rows
  // are not written and their live bytes stay 0 (cleared before the launch), so
  // the per-record sums skip them.  (About 4 in 5 pairs at 1M Gaussians:
  // writing zero rows at their scattered emission positions cost more than the
  // rest of the walk's stores.)

  // Starting state at the chunk's end: the final one when the walk ends in
  // this chunk, else the forward's record at ce (transmittance there, and the
  // colour composited after it, which gives the dL/dC-weighted colour behind)
  // for the pixels that still composite after ce; the others keep the final
  // state.  With forward chunking the record holds the colour composited
  // after ce within its forward chunk; the later chunks' colour is added.
  if (ce < wlim) {
    const int tpx = 1 << (a.log2_tw + a.log2_th);
    const float4* st = a.state + (int64_t)(ce >> lg) * tpx;
    const float4* sf = nullptr;
    if (a.log2_fchunk < 31) {
      const int lf = a.log2_fchunk;
      const uint64_t nxt = (uint64_t)tc.start + ((((ce - tc.start) >> lf) + 1) << lf);  // next forward boundary
      if (nxt < (uint64_t)tc.end) sf = a.fsuf + (int64_t)(nxt >> lf) * tpx;
    }
    const int rel = (int)(ce - tc.start);
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
      if (lc[p] > rel) {
        const float4 v = get4<L2>(st + threadIdx.x * PPT + p);
        float c0 = v.y, c1 = v.z, c2 = v.w;
        if (sf) {
          const float4 w = sf[threadIdx.x * PPT + p];
          c0 += w.x;
          c1 += w.y;
          c2 += w.z;
        }
        T[p] = v.x;
        RdL[p] = RdL[p] + (c0 * g0[p] + c1 * g1[p] + c2 * g2[p]);
      }
    }
  }

  const uint32_t cstart = (uint32_t)cs;
  const uint32_t wend = (uint32_t)min(ce, wlim);
  for (uint32_t be = wend; be > cstart;) {
    const uint32_t bs = (be - cstart > (uint32_t)batch) ? be - batch : cstart;
    const int cnt = (int)(be - bs);
    if (CULL) {
      // live pixels: those with an entry of this batch before their last contributor
      bool live[PPT];
#pragma unroll
      for (int p = 0; p < PPT; ++p) live[p] = lc[p] > (int)(bs - tc.start);
      const Box b = live_box<PPT>(px, py, live);
      if (lane == 0) s_box[wave] = b;
      __syncthreads();
    }
    for (int i = threadIdx.x; i < cnt; i += nthreads) {
      const uint32_t rec = a.ids[bs + i];
      const float4 ra = a.splats[(size_t)rec * 3 + 0];
      const float4 rb = a.splats[(size_t)rec * 3 + 1];
      s_e[i] = a.pair_index[bs + i];
      s_a[i] = staged_a(ra);
      s_b[i] = staged_b(rb);
      s_c[i] = a.splats[(size_t)rec * 3 + 2];
      if (CULL) s_mask[i] = (uint8_t)footprint_mask(ra, rb, nwaves, s_box);
    }
    for (int i = threadIdx.x; i < nwaves * batch * GS_GRAD_FLOATS; i += nthreads) s_part[i] = 0.0f;
    __syncthreads();
    const int nchunks = (cnt + kWave - 1) / kWave;
    for (int c = nchunks - 1; c >= 0; --c) {
      uint64_t m = chunk_bits<CULL>(s_mask, c, cnt, wave, lane);
      if (m == 0) continue;
      // one staged record: per-pixel partials, then the wave's sums into LDS
      auto grad = [&](int j, const float4& ra, const float4& rb, const float4& rc) {
        const int jr = (int)(bs - tc.start) + j;                   // index within the tile's list
        const float hb = 0.5f * ra.w;                              // staged b / 2 = k B
        float x[GS_GRAD_FLOATS] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};  // u v A B C o' r g b
        bool any = false;
#pragma unroll
        for (int p = 0; p < PPT; ++p) {
          // branch-free: lanes that do not composite this splat add exact zeros
          Eval e;
          const bool inside = eval_splat_all(px[p], py[p], ra.x, ra.y, ra.z, ra.w, rb.x, rb.y, rb.z, &e);
          const bool use = jr < lc[p] && inside && !(e.alpha < kAlphaMin);
          any |= use;
          const float inv = __builtin_amdgcn_rcpf(1.0f - e.alpha);
          T[p] = use ? T[p] * inv : T[p];  // transmittance in front of this splat
          const float wgt = use ? e.alpha * T[p] : 0.0f;
          x[6] += wgt * g0[p];
          x[7] += wgt * g1[p];
          x[8] += wgt * g2[p];
          const float cd = rc.x * g0[p] + rc.y * g1[p] + rc.z * g2[p];
          const float dLda = use && !(e.raw > kAlphaMax) ? T[p] * cd - RdL[p] * inv : 0.0f;
          RdL[p] += cd * wgt;
          x[5] += e.G * dLda;
          // m = alpha dL/dalpha = -2 dL/dq; the constant factors of the conic and
          // position gradients are applied once, after the wave's sums (kGradScale)
          const float m = e.alpha * dLda;
          x[2] += m * e.dx * e.dx;
          x[3] += m * e.dx * e.dy;
          x[4] += m * e.dy * e.dy;
          x[0] += m * (ra.z * e.dx + hb * e.dy);
          x[1] += m * (hb * e.dx + rb.x * e.dy);
        }
        if (__ballot(any) != 0) {  // wave-uniform: the whole wave takes part
          const float v = reduce_scatter9(x, b2, b3);
          if (writer) s_part[(wave * batch + j) * GS_GRAD_FLOATS + my_e] = v * escale;
        }
      };
      // two register sets in turn: the next record loads while this one is reduced
      int j0 = c * kWave + (63 - __builtin_clzll(m));  // back to front
      m &= ~(1ull << (j0 - c * kWave));
      float4 a0 = s_a[j0], b0 = s_b[j0], c0 = s_c[j0];
      for (;;) {
        const bool more1 = m != 0;
        const int j1 = more1 ? c * kWave + (63 - __builtin_clzll(m)) : j0;
        m &= ~(1ull << (j1 - c * kWave));
        const float4 a1 = s_a[j1], b1 = s_b[j1], c1 = s_c[j1];
        __builtin_amdgcn_sched_barrier(0);  // keep those loads ahead of this record's work
        grad(j0, a0, b0, c0);
        if (!more1) break;
        const bool more2 = m != 0;
        j0 = more2 ? c * kWave + (63 - __builtin_clzll(m)) : j1;
        m &= ~(1ull << (j0 - c * kWave));
        a0 = s_a[j0], b0 = s_b[j0], c0 = s_c[j0];
        __builtin_amdgcn_sched_barrier(0);
        grad(j1, a1, b1, c1);
        if (!more2) break;
      }
    }
    __syncthreads();
    // fixed-order sum over the waves, one store per (pair, attribute)
    for (int i = threadIdx.x; i < cnt * GS_GRAD_FLOATS; i += nthreads) {
      const int j = i / GS_GRAD_FLOATS, k = i - j * GS_GRAD_FLOATS;
      float v = s_part[j * GS_GRAD_FLOATS + k];
      for (int w = 1; w < nwaves; ++w) v += s_part[(w * batch + j) * GS_GRAD_FLOATS + k];
      grad_pair[(size_t)s_e[j] * GS_GRAD_FLOATS + k] = v;
      if (k == 0) a.pair_live[s_e[j]] = 1;
    }
    __syncthreads();
    be = bs;
  }
}

template <int PPT, bool CULL>
__global__ __launch_bounds__(256) void render_bwd_kernel(RenderArgs a, ViewTable vt, const float* __restrict__ T_final,
                                                         const int32_t* __restrict__ last_in,
                                                         const float* __restrict__ dL_dimage,
                                                         float* __restrict__ grad_pair) {
  extern __shared__ __align__(16) unsigned char smem[];
  LossIn loss;
  loss.dL_dimage = dL_dimage;
  loss.image = loss.target = nullptr;
  loss.dL_out = nullptr;
  bwd_item<PPT, CULL, false>(a, vt, T_final, last_in, loss, grad_pair, (int64_t)blockIdx.x, smem);
}

// Backward work list of the one-launch walks.  Each tile contributes its first
// chunk and one item per boundary (start + k 2^log2_chunk, k >= 1, whether or
// not the forward walk reaches it: a chunk past the walk then finds nothing to
// do).  Tiles are grouped by the bit length of their list length and the groups
// laid out lightest first: a tile's backward items are then taken about when its
// forward walk ends, and the deepest lists' items, whose forward walks end last,
// come last (an item taken before its tile's forward walk has ended holds its
// workgroup slot while it waits).  An entry is a render_bwd_kernel item number
// with the schedule off: a boundary chunk is its slot, tile t's first chunk
// nslots + t.  The count pass also records each boundary's owner.
// hist: [0, 64) items per group, [64, 128) write positions, [128] the total.
__device__ __forceinline__ int list_group(uint32_t len) { return len ? 32 - __clz(len) : 0; }

__device__ __forceinline__ uint32_t list_items(uint32_t len, int lg) {
  return (uint64_t)len > (1ull << lg) ? (uint32_t)(((uint64_t)len - 1) >> lg) + 1u : 1u;
}

__device__ __forceinline__ uint32_t list_len(const RenderArgs& a, int64_t t) {
  return *a.status == 0 ? a.ranges[2 * t + 1] - a.ranges[2 * t] : 0u;
}

__global__ __launch_bounds__(256) void list_count_kernel(RenderArgs a, int64_t tiles, uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[64];
  if (threadIdx.x < 64) h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < tiles) {
    const uint32_t len = list_len(a, t);
    const int lg = a.log2_chunk;
    const uint64_t start = a.ranges[2 * t];
    for (uint64_t q = start + (1ull << lg); q < start + len; q += 1ull << lg) a.slot_owner[q >> lg] = (uint32_t)t;
    atomicAdd(&h[list_group(len)], list_items(len, lg));
  }
  __syncthreads();
  if (threadIdx.x < 64 && h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], h[threadIdx.x]);
}

__global__ void list_scan_kernel(uint32_t* __restrict__ hist) {
  if (threadIdx.x != 0) return;
  uint32_t run = 0;
  for (int g = 0; g < 64; ++g) {
    hist[64 + g] = run;
    run += hist[g];
  }
  hist[128] = run;
}

__global__ __launch_bounds__(256) void list_scatter_kernel(RenderArgs a, int64_t tiles, uint32_t* __restrict__ hist,
                                                           uint32_t* __restrict__ list) {
  // offsets within the block per group (LDS), one global reservation per group and block
  __shared__ uint32_t h[64], base[64];
  if (threadIdx.x < 64) h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int lg = a.log2_chunk;
  int g = 0;
  uint32_t len = 0, n = 0, off = 0;
  if (t < tiles) {
    len = list_len(a, t);
    g = list_group(len);
    n = list_items(len, lg);
    off = atomicAdd(&h[g], n);
  }
  __syncthreads();
  if (threadIdx.x < 64 && h[threadIdx.x]) base[threadIdx.x] = atomicAdd(&hist[64 + threadIdx.x], h[threadIdx.x]);
  __syncthreads();
  if (t >= tiles) return;
  uint32_t* out = list + base[g] + off;
  out[0] = (uint32_t)(a.nslots + t);
  const uint64_t start = a.ranges[2 * t];
  for (uint32_t k = 1; k < n; ++k) out[k] = (uint32_t)((start + ((uint64_t)k << lg)) >> lg);
}

// Polls (at most kWaitPolls times, sleeping about 2000 cycles between polls)
// until the flag is set; its value, or 0 if it never was (after about a second).
constexpr int kWaitPolls = 1 << 20;
__device__ __forceinline__ uint32_t wait_flag(const uint32_t* flag) {
  for (int i = 0; i < kWaitPolls; ++i) {
    const uint32_t v = __hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (v != 0u) return v;
    __builtin_amdgcn_s_sleep(32);
  }
  return 0u;
}

// Forward and backward walks in one launch, for the mean-squared-error loss
// (the loss gradient of a pixel needs only that pixel).  Each workgroup takes
// the next work item from a ticket: first every tile's forward walk in the
// heaviest-first schedule, then the backward work list (lightest lists first,
// see list_count_kernel).  A forward item sets its tile's flag once the image,
// T_final, last_contrib and chunk states of the tile are written; a backward
// item waits for its tile's flag, which holds 1 + the tile's largest
// last_contrib (a boundary chunk past it then leaves at once).  The flags it
// waits for belong to items taken earlier, which wait for nothing, so every
// wait ends (a wait that outlives its poll limit gives up and makes the item's
// gradients NaN instead of blocking).
// The backward items of finished tiles run while the deepest tiles' forward
// walks are still going.  sync: [total_tiles] flags, the ticket, all zero at
// launch, then the list's counts (kListHist words) and the list.
// At one pixel a thread the kernel is held to 80 registers (six waves per SIMD,
// as many as the backward's LDS allows).
template <int PPT, bool CULL>
__global__ __launch_bounds__(256, PPT == 1 ? 6 : 1) void render_fused_kernel(RenderArgs a, ViewTable vt,
                                                                             float* __restrict__ image,
                                                                             float* __restrict__ T_final,
                                                                             int32_t* __restrict__ last, LossIn loss,
                                                                             float* __restrict__ grad_pair,
                                                                             uint32_t* __restrict__ sync) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ uint32_t s_ticket;
  __shared__ uint32_t s_flag;
  __shared__ int s_wmax[4];
  const int64_t ntiles = vt.total_tiles;
  if (threadIdx.x == 0) s_ticket = atomicAdd(sync + ntiles, 1u);
  __syncthreads();
  const int64_t q = s_ticket;
  if (q < ntiles) {
    // forward walks issue ahead of the backward waves that share their SIMD:
    // the deepest lists' forward walks are the launch's critical path
    __builtin_amdgcn_s_setprio(3);
    int my_max = fwd_item<PPT, CULL, kFull, true>(
        a, vt, image, T_final, last, q, (float4(*)[3][kHalves * kWave])smem,
        (uint32_t(*)[kHalves * kWave])(smem + sizeof(float4) * 4 * 3 * kHalves * kWave));
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) my_max = max(my_max, __shfl_xor(my_max, o, kWave));
    if ((threadIdx.x & (kWave - 1)) == 0) s_wmax[threadIdx.x / kWave] = my_max;
    // every thread's coherent stores of image, T_final, last_contrib and
    // states have been acknowledged before the flag is set
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
      int m = 0;
      for (int w = 0; w < (int)blockDim.x / kWave; ++w) m = max(m, s_wmax[w]);
      const int gtile = a.order ? (int)a.order[q] : (int)q;
      // the flag: 1 + the largest last_contrib of the tile
      __hip_atomic_store(sync + gtile, (uint32_t)m + 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    return;
  }
  const uint32_t* hist = sync + ntiles + 1;
  const int64_t qb = q - ntiles;
  if (qb >= (int64_t)hist[128]) return;  // past the list (the grid is sized for the most items)
  const int64_t item = hist[kListHist + qb];
  RenderArgs ab = a;
  ab.order = nullptr;  // first chunks are numbered by tile
  if (threadIdx.x == 0) {
    int gtile = -1;
    if (item < a.nslots) {
      const uint32_t owner = a.slot_owner[item];
      if (owner < (uint32_t)ntiles) gtile = (int)owner;
    } else {
      gtile = (int)(item - a.nslots);
    }
    s_flag = gtile < 0 ? 1u : wait_flag(sync + gtile);
  }
  __syncthreads();  // the tile's values are then read with coherent loads
  // a flag never seen set: the item's loss gradient, hence its gradients, are NaN
  const uint32_t f = s_flag;
  bwd_item<PPT, CULL, true>(ab, vt, T_final, last, loss, grad_pair, item, smem, f != 0u, f != 0u ? (int)(f - 1u) : -1);
}

static int tile_threads(const RenderArgs& a) { return (1 << (a.log2_tw + a.log2_th)) / a.ppt; }

// Work items [item_base, item_base + items) of one walk launch.
template <int PPT, int MODE>
static void walk(const RenderArgs& a, const ViewTable& vt, float* image, float* T_final, int32_t* last,
                 int64_t item_base, int64_t items, hipStream_t s) {
  if (items <= 0) return;
  const int nt = tile_threads(a);
  const dim3 grid((unsigned)items), block((unsigned)nt);
  if (a.cull)
    hipLaunchKernelGGL((render_fwd_kernel<PPT, true, MODE>), grid, block, 0, s, a, vt, image, T_final, last,
                       item_base);
  else
    hipLaunchKernelGGL((render_fwd_kernel<PPT, false, MODE>), grid, block, 0, s, a, vt, image, T_final, last,
                       item_base);
}

template <int PPT>
static void fwd_ppt(const RenderArgs& a, const ViewTable& vt, float* image, float* T_final, int32_t* last,
                    hipStream_t s) {
  if (a.nfslots > 0)
    hipLaunchKernelGGL(fwd_mark_kernel, dim3((unsigned)((vt.total_tiles + 255) / 256)), dim3(256), 0, s, a,
                       vt.total_tiles);
  walk<PPT, kFull>(a, vt, image, T_final, last, a.nfslots, vt.total_tiles, s);  // every tile's first chunk
  if (a.nfslots > 0) {
    walk<PPT, kTPass>(a, vt, nullptr, nullptr, nullptr, 0, a.nfslots, s);  // products of chunks 1 .. m-2
    walk<PPT, kFull>(a, vt, image, T_final, last, 0, a.nfslots, s);       // chunks 1 .. m-1
    hipLaunchKernelGGL((fwd_combine_kernel<PPT>), dim3((unsigned)vt.total_tiles), dim3((unsigned)tile_threads(a)), 0,
                       s, a, vt, image, T_final, last);
  }
}

template <int PPT>
static void count_ppt(const RenderArgs& a, const ViewTable& vt, hipStream_t s) {
  walk<PPT, kCount>(a, vt, nullptr, nullptr, nullptr, 0, vt.total_tiles, s);
}

template <int PPT>
static void bwd_ppt(const RenderArgs& a, const ViewTable& vt, const float* T_final, const int32_t* last,
                    const float* dL, float* grad_pair, hipStream_t s) {
  const int nt = tile_threads(a);
  // chunk items first, then one item per tile
  const dim3 grid((unsigned)(a.nslots + vt.total_tiles)), block((unsigned)nt);
  const size_t sh = lds_bytes(bwd_batch(a.batch, nt / kWave), nt / kWave, true);
  if (a.cull)
    hipLaunchKernelGGL((render_bwd_kernel<PPT, true>), grid, block, sh, s, a, vt, T_final, last, dL, grad_pair);
  else
    hipLaunchKernelGGL((render_bwd_kernel<PPT, false>), grid, block, sh, s, a, vt, T_final, last, dL, grad_pair);
}

hipError_t launch_render_fwd(const RenderArgs& a, const ViewTable& vt, float* image, float* T_final,
                             int32_t* last_contrib, hipStream_t s) {
  if (vt.total_tiles == 0) return hipSuccess;
  hipError_t e = launch_fill_u32(a.slot_owner, a.nslots, 0xffffffffu, s);  // no boundary recorded yet
  if (e != hipSuccess) return e;
  if (a.nfslots > 0 && (e = launch_fill_u32(a.fslot_owner, a.nfslots, 0xffffffffu, s)) != hipSuccess) return e;
  switch (a.ppt) {
    case 1: fwd_ppt<1>(a, vt, image, T_final, last_contrib, s); break;
    case 2: fwd_ppt<2>(a, vt, image, T_final, last_contrib, s); break;
    default: fwd_ppt<4>(a, vt, image, T_final, last_contrib, s); break;
  }
  return hipGetLastError();
}

hipError_t launch_count_hits(const RenderArgs& a, const ViewTable& vt, hipStream_t s) {
  if (vt.total_tiles == 0) return hipSuccess;
  switch (a.ppt) {
    case 1: count_ppt<1>(a, vt, s); break;
    case 2: count_ppt<2>(a, vt, s); break;
    default: count_ppt<4>(a, vt, s); break;
  }
  return hipGetLastError();
}

template <int PPT>
static void fused_ppt(const RenderArgs& a, const ViewTable& vt, float* image, float* T_final, int32_t* last,
                      const LossIn& loss, float* grad_pair, uint32_t* sync, hipStream_t s) {
  const int nt = tile_threads(a);
  const size_t bwd_sh = lds_bytes(bwd_batch(a.batch, nt / kWave), nt / kWave, true);
  const size_t fwd_sh = (sizeof(float4) * 4 * 3 + sizeof(uint32_t) * 4) * kHalves * kWave;
  const size_t sh = bwd_sh > fwd_sh ? bwd_sh : fwd_sh;
  // forward items, then at most one backward item per tile and one per boundary slot
  const dim3 grid((unsigned)(2 * vt.total_tiles + a.nslots)), block((unsigned)nt);
  if (a.cull)
    hipLaunchKernelGGL((render_fused_kernel<PPT, true>), grid, block, sh, s, a, vt, image, T_final, last, loss,
                       grad_pair, sync);
  else
    hipLaunchKernelGGL((render_fused_kernel<PPT, false>), grid, block, sh, s, a, vt, image, T_final, last, loss,
                       grad_pair, sync);
}

hipError_t launch_render_fused(const RenderArgs& a, const ViewTable& vt, float* image, float* T_final,
                               int32_t* last_contrib, const float* target, const float* scale, float* dL_out,
                               float* grad_pair, uint32_t* sync, hipStream_t s) {
  if (vt.total_tiles == 0) return hipSuccess;
  if (a.nfslots != 0) return hipErrorInvalidValue;  // forward chunking runs as separate launches
  LossIn loss;
  loss.dL_dimage = nullptr;
  loss.image = image;
  loss.target = target;
  loss.dL_out = dL_out;
  for (int v = 0; v < GS_MAX_VIEWS; ++v) loss.scale[v] = v < vt.nviews ? scale[v] : 0.0f;
  hipError_t e = launch_fill_u32(a.slot_owner, a.nslots, 0xffffffffu, s);
  if (e == hipSuccess) e = launch_fill_u32(sync, vt.total_tiles + 1 + 64, 0u, s);  // flags, ticket, list counts
  if (e != hipSuccess) return e;
  uint32_t* hist = sync + vt.total_tiles + 1;
  const dim3 tgrid((unsigned)((vt.total_tiles + 255) / 256));
  hipLaunchKernelGGL(list_count_kernel, tgrid, dim3(256), 0, s, a, (int64_t)vt.total_tiles, hist);
  hipLaunchKernelGGL(list_scan_kernel, dim3(1), dim3(64), 0, s, hist);
  hipLaunchKernelGGL(list_scatter_kernel, tgrid, dim3(256), 0, s, a, (int64_t)vt.total_tiles, hist,
                     hist + kListHist);
  switch (a.ppt) {
    case 1: fused_ppt<1>(a, vt, image, T_final, last_contrib, loss, grad_pair, sync, s); break;
    case 2: fused_ppt<2>(a, vt, image, T_final, last_contrib, loss, grad_pair, sync, s); break;
    default: fused_ppt<4>(a, vt, image, T_final, last_contrib, loss, grad_pair, sync, s); break;
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
