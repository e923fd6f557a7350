// Kernel argument structs and launch wrappers of libgs (host + device).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gs_common.h"

namespace gs {

struct ProjectArgs {
  const float* means;
  const float* log_scales;
  const float* quats;
  const float* opacity_logits;
  const float* sh_dc;
  const float* sh_rest;
  const float* mask_logits;
  const float* sh_mask_logits;
  int64_t n;
  float mask_thr;     // logit(mask_eps), rounded down to float
  float sh_mask_thr;  // logit(sh_mask_eps), rounded down to float
  float near_plane;
  float inv_tw, inv_th;
  float4* splats;
  uint32_t* tiles_touched;
};

struct RenderArgs {
  const float4* splats;
  const uint32_t* ids;
  const uint32_t* pair_index;
  uint8_t* pair_live;     // backward: [capacity] 1 where the pair's gradient row was written
  const uint32_t* ranges;
  const uint32_t* order;  // tile schedule (NULL: tile-id order)
  const int32_t* status;
  int32_t log2_tw, log2_th;
  int32_t log2_sw, log2_sh;  // sub-tile (one per wave) width and height
  int32_t log2_sx;           // sub-tiles along x
  int32_t batch;
  int32_t ppt;
  int32_t cull;
  float bg[3];
  // per-chunk pixel states written by the forward, read by the backward:
  // boundary position q = start + k * 2^log2_chunk (k >= 1) of a tile's list
  // owns slot q >> log2_chunk; slot_owner[slot] = global tile, state[slot][pixel]
  // = (T, colour composited after q)
  int32_t log2_chunk;
  int64_t nslots;
  uint32_t* slot_owner;
  float4* state;
  // hit counting (Eq. 4): per-Gaussian counters, n Gaussians per view
  uint32_t* hits;
  int64_t n;
  // forward chunking: lists longer than 2^log2_fchunk entries (31: off) are
  // walked in chunks by separate workgroups.  Forward boundary q = start + kF
  // (k >= 1) owns slot q >> log2_fchunk: fslot_owner[slot] = global tile;
  // fprod[slot][pixel] = product of (1 - alpha) over the chunk ending at q;
  // fres/flast[slot] = (colour, final T) / last index of the chunk ending at
  // q, and at [nfslots + slot] those of a list's last chunk starting at q;
  // fsuf[slot] = colour composited from q on (read by the backward).
  int32_t log2_fchunk;
  int64_t nfslots;
  uint32_t* fslot_owner;
  float* fprod;
  float4* fres;
  int32_t* flast;
  float4* fsuf;
};

struct BinOut {
  uint64_t* keys;
  uint32_t* ids;
  uint32_t* pair_index;
  uint32_t* offsets;
  uint32_t* ranges;
  uint32_t* order;
  uint32_t* count;
  int32_t* status;
};

constexpr int kRecPlanes = 9;

struct ProjectBwdArgs {
  ProjectArgs p;                   // forward inputs (outputs unused)
  const float* grad_pair;          // [K][9], emission order
  const uint32_t* tiles_touched;   // [V*n]
  const uint32_t* offsets;         // [V*n] first emission position of each record
  const uint8_t* pair_live;        // [K] 1 where the walk wrote the pair's row (others count as zero)
  const int32_t* status;
  float* rec;                      // [kRecPlanes][rec_stride] per record: sums of the (u, v, A, B, C, o')
                                   // gradients, then the colour term of the mean gradient
  int64_t rec_stride;              // V*n rounded up to 64
  float* g_means;
  float* g_log_scales;
  float* g_quats;
  float* g_opacity_logits;
  float* g_sh_dc;
  float* g_sh_rest;
  float* g_mask_logits;
  float* g_sh_mask_logits;
  float* g_mean2d;
  int32_t assign;                  // 1: write the parameter gradients (zeros where none), 0: add them
};

// Views of an image call (loss: 32 x 32 tiles; target blur: 16 x 16): per
// view its size, tile grid, pixel offset (views concatenated, each [3][H][W])
// and first workgroup; the loss window's taps.
constexpr int kLossTile = 32;
constexpr int kBlurTile = 16;
struct LossView {
  int32_t W, H, TX, TY;
  int64_t pix_off;
  int32_t block_off;
};
struct LossViews {
  LossView v[GS_MAX_VIEWS];
  int32_t nviews;
  int32_t total_blocks;
  float g[11];  // normalised Gaussian taps of the 11 x 11 window's 1-D factor
};

// Workgroup b of an image call: its view, colour plane and 16 x 16 tile.
struct LossTile {
  int view, plane, tx, ty;
};

__device__ __forceinline__ LossTile loss_tile(const LossViews& lv, int b) {
  LossTile t;
  int v = 0;
  while (v + 1 < lv.nviews && b >= lv.v[v + 1].block_off) ++v;
  const LossView& q = lv.v[v];
  const int lb = b - q.block_off;
  const int per_plane = q.TX * q.TY;
  t.view = v;
  t.plane = lb / per_plane;
  const int r = lb - t.plane * per_plane;
  t.ty = r / q.TX;
  t.tx = r - t.ty * q.TX;
  return t;
}

// Target blur: the views' 16 x 16 tiles, radius r = (k - 1) / 2 and the k taps.
constexpr int kMaxBlurRadius = 15;
struct BlurArgs {
  LossViews views;
  int32_t r;
  float g[2 * kMaxBlurRadius + 1];
};

// Mean squared error gradient: per view the end of its elements and the scale.
struct L2Args {
  int64_t end[GS_MAX_VIEWS];  // exclusive end of view v's 3 H W elements
  float scale[GS_MAX_VIEWS];  // 2 / (3 H W mean_views)
  int32_t nviews;
};
hipError_t launch_l2_grad(const float* image, const float* target, float* dL, const L2Args& a, hipStream_t s);
// Forward and backward walks in one launch with the mean-squared-error gradient
// dL = scale[v] (image - target) computed inline (render.hip).  Needs forward
// chunking off; pair_live cleared by the caller; sync: fused_sync_words u32
// (tile flags, the ticket, kListHist counts of the backward work list, the list).
constexpr int kListHist = 129;
inline int64_t fused_sync_words(int64_t total_tiles, int64_t nslots) {
  return total_tiles + 1 + kListHist + total_tiles + nslots;
}
hipError_t launch_render_fused(const RenderArgs& a, const ViewTable& vt, float* image, float* T_final,
                               int32_t* last_contrib, const float* target, const float* scale, float* dL_out,
                               float* grad_pair, uint32_t* sync, hipStream_t s);

// Target resize: per view the input and output sizes and pixel offsets.
struct ResizeView {
  int32_t W, H, Wo, Ho;
  int64_t in_off, out_off;
  float inv_area;  // 1 / (W H)
};
struct ResizeArgs {
  ResizeView v[GS_MAX_VIEWS];
  int32_t nviews;
  int64_t total_out;  // 3 * sum of W' H'
};

hipError_t launch_blur(const float* in, float* out, const BlurArgs& b, hipStream_t s);
hipError_t launch_resize(const float* in, float* out, const ResizeArgs& a, hipStream_t s);

hipError_t launch_loss(const LossViews& lv, const float* image, const float* target, float lambda, float* loss,
                       float* dL, float* dmap, float* bsum, double* per_view, hipStream_t s);

hipError_t launch_mask_loss(const float* m, const float* msh, int64_t n, int deg, float lam_m, float lam_sh,
                            float* gm, float* gsh, float* loss, float* bsum, hipStream_t s);

// Radix-select state of the volume quantile (significance score).
struct SelectState {
  uint32_t prefix;  // key bits chosen so far
  uint32_t rank;    // rank still wanted among the keys matching the prefix
  uint32_t pad[2];
  uint32_t hist[256];
};

hipError_t launch_significance(const float* log_scales, const float* opacity_logits, const float* mask_logits,
                               float mask_thr, const uint32_t* hits, int64_t n, uint32_t rank, SelectState* st,
                               float* score, hipStream_t s);

// Workspace carve-up of gs_bin_sort / gs_render_bwd.
struct SortPlan {
  int64_t nrec;             // V * n
  uint64_t capacity;        // pair capacity
  int64_t scan_blocks;      // records / 1024
  int64_t rec_sort_blocks;  // records / 4096 (depth sort of the visible records)
  int64_t sort_blocks;      // capacity / 4096 (tile sort of the pairs)
  int tile_passes;          // 8-bit passes over ceil(log2 #tiles) tile bits
};

hipError_t launch_project(const ProjectArgs& a, const ViewTable& vt, int deg, hipStream_t s);

hipError_t launch_bin_sort(const SortPlan& plan, const float4* splats, const uint32_t* tiles_touched, int64_t n,
                           const ViewTable& vt, float inv_tw, float inv_th, const BinOut& out, uint64_t capacity,
                           void* ws, hipStream_t s);

hipError_t launch_render_fwd(const RenderArgs& a, const ViewTable& vt, float* image, float* T_final,
                             int32_t* last_contrib, hipStream_t s);

hipError_t launch_count_hits(const RenderArgs& a, const ViewTable& vt, hipStream_t s);

hipError_t launch_render_bwd(const RenderArgs& a, const ViewTable& vt, const float* T_final,
                             const int32_t* last_contrib, const float* dL_dimage, float* grad_pair, hipStream_t s);

hipError_t launch_project_bwd(const ProjectBwdArgs& a, const ViewTable& vt, int deg, hipStream_t s);

hipError_t launch_fill_u32(uint32_t* p, int64_t count, uint32_t value, hipStream_t s);

size_t bin_sort_ws_bytes(const SortPlan& plan);

}  // namespace gs
