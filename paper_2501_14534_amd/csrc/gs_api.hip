// Host side of the libgs C ABI: argument validation, per-view constant
// tables, workspace carve-up and kernel launches on the caller's stream.
// Nothing here allocates, frees, synchronises or reads device memory.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>

#include "gs_api.h"
#include "kernels.h"

using namespace gs;

// Scratch of gs_mask_loss_noalloc, the entry point for callers that cannot
// allocate: the per-workgroup partial sums of the mask terms, two floats per
// 256 Gaussians, for at most kNoAllocMaxGaussians Gaussians (512 KiB).  Each
// device holds its own copy for the life of the process; host code reaches it
// only through the address hipGetSymbolAddress returns on that device.
constexpr int64_t kNoAllocMaxGaussians = (int64_t)1 << 24;
constexpr size_t kScratchFloats = 2 * (size_t)(kNoAllocMaxGaussians / 256);
static __device__ __align__(256) float scratch[kScratchFloats];

namespace {

bool pow2(int x) { return x > 0 && (x & (x - 1)) == 0; }

int ilog2(int x) {
  int r = 0;
  while ((1 << r) < x) ++r;
  return r;
}

int device_ok() {
  static int cached[64] = {0};  // 0 unknown, 1 gfx950, -1 other
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return GS_E_HIP;
  if (cached[dev] == 0) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return GS_E_HIP;
    cached[dev] = std::strncmp(prop.gcnArchName, "gfx950", 6) == 0 ? 1 : -1;
  }
  return cached[dev] == 1 ? GS_OK : GS_E_UNSUPPORTED;
}

// Device address of `scratch` on the current device, looked up once per device
// with that device current; NULL if the lookup fails.
float* scratch_on_current_device() {
  static std::mutex mu;
  static float* addr[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
    addr[dev] = (float*)p;
  }
  return addr[dev];
}

// logit(eps) rounded down to a float, so that for every float m:
// (m > thr)  <=>  (m > logit(eps))  <=>  (sigmoid(m) > eps) in exact arithmetic.
bool mask_threshold(float eps, float* thr) {
  if (!(eps > 0.0f && eps < 1.0f)) return false;
  const double L = std::log((double)eps / (1.0 - (double)eps));
  float f = (float)L;
  if ((double)f > L) f = std::nextafter(f, -INFINITY);
  *thr = f;
  return true;
}

bool opts_ok(const gs_opts* o) {
  if (!o) return false;
  if (!pow2(o->tile_w) || !pow2(o->tile_h)) return false;
  const int px = o->tile_w * o->tile_h;
  if (px < 64 || px > 1024) return false;
  if (o->pixels_per_thread != 1 && o->pixels_per_thread != 2 && o->pixels_per_thread != 4) return false;
  if (px % (64 * o->pixels_per_thread) != 0) return false;
  if (px / o->pixels_per_thread > 256) return false;  // render kernels run <= 256 threads per tile
  if (o->batch_depth < 1 || o->batch_depth > GS_MAX_BATCH) return false;
  if (o->subtile_cull != 0 && o->subtile_cull != 1) return false;
  if (o->bwd_chunk != 0 && (!pow2(o->bwd_chunk) || o->bwd_chunk < 16 || o->bwd_chunk > (1 << 20))) return false;
  if (o->fwd_chunk != 0 && (!pow2(o->fwd_chunk) || o->fwd_chunk < 64 || o->fwd_chunk > (1 << 24))) return false;
  if (!std::isfinite(o->lowpass) || o->lowpass < 0.0f) return false;
  if (o->lowpass_progressive != 0 && o->lowpass_progressive != 1) return false;
  if (!std::isfinite(o->near_plane) || !(o->near_plane > 0.0f)) return false;  // depths > 0 order as bits
  if (!(o->tan_clamp > 0.0f)) return false;
  for (int c = 0; c < 3; ++c)
    if (!std::isfinite(o->bg[c])) return false;
  return true;
}

bool view_table(const gs_camera* cams, int32_t V, const gs_opts* o, ViewTable* vt, int64_t* total_pixels) {
  if (!cams || V < 1 || V > GS_MAX_VIEWS || !opts_ok(o)) return false;
  std::memset(vt, 0, sizeof(*vt));
  int64_t to = 0, po = 0;
  for (int v = 0; v < V; ++v) {
    const gs_camera& c = cams[v];
    if (c.width <= 0 || c.height <= 0 || !(c.fx > 0.0f) || !(c.fy > 0.0f)) return false;
    for (int k = 0; k < 9; ++k)
      if (!std::isfinite(c.R[k])) return false;
    for (int k = 0; k < 3; ++k)
      if (!std::isfinite(c.t[k])) return false;
    ViewArgs& a = vt->v[v];
    std::memcpy(a.R, c.R, sizeof(a.R));
    std::memcpy(a.t, c.t, sizeof(a.t));
    a.fx = c.fx, a.fy = c.fy, a.cx = c.cx, a.cy = c.cy;
    for (int j = 0; j < 3; ++j)
      a.campos[j] = (float)-((double)c.R[j] * c.t[0] + (double)c.R[3 + j] * c.t[1] + (double)c.R[6 + j] * c.t[2]);
    a.limx = (float)((double)o->tan_clamp * 0.5 * c.width / c.fx);
    a.limy = (float)((double)o->tan_clamp * 0.5 * c.height / c.fy);
    a.W = c.width, a.H = c.height;
    a.TX = (c.width + o->tile_w - 1) / o->tile_w;
    a.TY = (c.height + o->tile_h - 1) / o->tile_h;
    if (a.TX > 65535 || a.TY > 65535) return false;  // tile rectangles are packed as 16-bit sizes
    a.tile_off = (int32_t)to;
    a.pix_off = (int32_t)po;
    a.lowpass = o->lowpass;
    to += (int64_t)a.TX * a.TY;
    po += (int64_t)c.width * c.height;
    if (to >= (1ll << 31) || 3 * po >= (1ll << 31)) return false;
  }
  vt->nviews = V;
  vt->total_tiles = (int32_t)to;
  if (total_pixels) *total_pixels = po;
  return true;
}

// Per-view low-pass of a call on n Gaussians: with progressive scaling
// (Sec. 3.2.4) s_v = max(lowpass, W_v H_v / (9 pi n)), so that each projected
// Gaussian covers at least 9 pi s_v, the share of the view that n of them fill.
void set_lowpass(ViewTable* vt, const gs_opts* o, int64_t n) {
  for (int v = 0; v < vt->nviews; ++v) {
    ViewArgs& a = vt->v[v];
    double s = o->lowpass;
    if (o->lowpass_progressive && n > 0) s = std::max(s, (double)a.W * (double)a.H / (9.0 * M_PI * (double)n));
    a.lowpass = (float)s;
  }
}

bool gaussians_ok(const gs_gaussians* g, ProjectArgs* a) {
  if (!g || g->n < 0 || g->n >= (1ll << 31) || g->sh_degree < 0 || g->sh_degree > 3) return false;
  if (g->n > 0 && (!g->means || !g->log_scales || !g->quats || !g->opacity_logits || !g->sh_dc)) return false;
  if (g->n > 0 && g->sh_degree > 0 && !g->sh_rest) return false;
  std::memset(a, 0, sizeof(*a));
  a->means = g->means, a->log_scales = g->log_scales, a->quats = g->quats;
  a->opacity_logits = g->opacity_logits, a->sh_dc = g->sh_dc;
  a->sh_rest = g->sh_degree > 0 ? g->sh_rest : nullptr;
  a->mask_logits = g->mask_logits;
  a->sh_mask_logits = g->sh_degree > 0 ? g->sh_mask_logits : nullptr;
  a->n = g->n;
  a->mask_thr = 0.f;
  a->sh_mask_thr = 0.f;
  if (g->mask_logits && !mask_threshold(g->mask_eps, &a->mask_thr)) return false;
  if (g->sh_mask_logits && g->sh_degree > 0 && !mask_threshold(g->sh_mask_eps, &a->sh_mask_thr)) return false;
  return true;
}

SortPlan sort_plan(int64_t n, int32_t V, int32_t total_tiles, uint64_t capacity) {
  SortPlan p;
  p.nrec = (int64_t)V * n;
  p.capacity = capacity;
  p.scan_blocks = (p.nrec + 1023) / 1024;
  p.rec_sort_blocks = (p.nrec + 4095) / 4096;
  p.sort_blocks = (int64_t)((capacity + 4095) / 4096);
  p.tile_passes = ((total_tiles > 1 ? ilog2(total_tiles) : 0) + 7) / 8;
  return p;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
bool aligned(const void* p, uintptr_t a) { return ((uintptr_t)p & (a - 1)) == 0; }

// Chunk length of the backward work items (2^31: one item per tile).
int log2_chunk(const gs_opts* o) { return o->bwd_chunk ? ilog2(o->bwd_chunk) : 31; }
int64_t chunk_slots(uint64_t capacity, const gs_opts* o) { return (int64_t)(capacity >> log2_chunk(o)) + 1; }
int log2_fchunk(const gs_opts* o) { return o->fwd_chunk ? ilog2(o->fwd_chunk) : 31; }
int64_t fchunk_slots(uint64_t capacity, const gs_opts* o) {
  return o->fwd_chunk ? (int64_t)(capacity >> log2_fchunk(o)) + 1 : 0;
}

// Per-chunk pixel states, after the backward's own regions in the workspace:
// slot owners [slots] u32, then states [slots][tile pixels] float4.
size_t state_owner_bytes(uint64_t capacity, const gs_opts* o) {
  return align256(sizeof(uint32_t) * (size_t)chunk_slots(capacity, o));
}
// Forward chunking: owners [fslots] u32, products [fslots][px] f32, results
// [2 fslots][px] float4 and [2 fslots][px] i32, suffix colours [fslots][px] float4.
struct FwdChunkWs {
  size_t owner, prod, res, last, suf, bytes;
};
FwdChunkWs fwd_chunk_ws(uint64_t capacity, const gs_opts* o) {
  const size_t fs = (size_t)fchunk_slots(capacity, o), px = (size_t)(o->tile_w * o->tile_h);
  FwdChunkWs w;
  w.owner = 0;
  w.prod = w.owner + align256(4 * fs);
  w.res = w.prod + align256(4 * fs * px);
  w.last = w.res + align256(16 * 2 * fs * px);
  w.suf = w.last + align256(4 * 2 * fs * px);
  w.bytes = w.suf + align256(16 * fs * px);
  return w;
}
size_t render_state_bytes(uint64_t capacity, const gs_opts* o) {
  return state_owner_bytes(capacity, o) +
         align256(16 * (size_t)chunk_slots(capacity, o) * (size_t)(o->tile_w * o->tile_h)) +
         (o->fwd_chunk ? fwd_chunk_ws(capacity, o).bytes : 0);
}

RenderArgs render_args(const gs_projected* p, const gs_binning* b, const gs_opts* o) {
  RenderArgs a;
  a.splats = (const float4*)p->splats;
  a.ids = b->ids;
  a.pair_index = b->pair_index;
  a.pair_live = nullptr;
  a.ranges = b->ranges;
  a.order = b->order;
  a.status = b->status;
  a.log2_tw = ilog2(o->tile_w);
  a.log2_th = ilog2(o->tile_h);
  // one sub-tile of 64 * ppt pixels per wave, as square as the tile allows (wider on ties)
  const int log2_waves = a.log2_tw + a.log2_th - 6 - ilog2(o->pixels_per_thread);
  int best = -1;
  for (int sx = 0; sx <= log2_waves; ++sx) {
    const int sw = a.log2_tw - sx, sh = a.log2_th - (log2_waves - sx);
    if (sw < 0 || sh < 0) continue;
    if (best < 0 || std::abs(sw - sh) < std::abs(a.log2_sw - a.log2_sh) ||
        (std::abs(sw - sh) == std::abs(a.log2_sw - a.log2_sh) && sw > a.log2_sw)) {
      best = sx;
      a.log2_sx = sx;
      a.log2_sw = sw;
      a.log2_sh = sh;
    }
  }
  a.batch = o->batch_depth;
  a.ppt = o->pixels_per_thread;
  a.cull = o->subtile_cull;
  for (int c = 0; c < 3; ++c) a.bg[c] = o->bg[c];
  a.log2_chunk = log2_chunk(o);
  a.nslots = chunk_slots(b->capacity, o);
  a.slot_owner = nullptr;
  a.state = nullptr;
  a.hits = nullptr;
  a.n = 0;
  a.log2_fchunk = log2_fchunk(o);
  a.nfslots = fchunk_slots(b->capacity, o);
  a.fslot_owner = nullptr;
  a.fprod = nullptr;
  a.fres = nullptr;
  a.flast = nullptr;
  a.fsuf = nullptr;
  return a;
}

int launched(hipError_t e) { return e == hipSuccess ? GS_OK : GS_E_HIP; }

bool binning_ok(const gs_binning* b, int64_t nrec) {
  if (!b || !b->ranges || !b->count || !b->status || b->capacity >= (1ull << 32)) return false;
  if (b->capacity > 0 && (!b->ids || !b->pair_index)) return false;
  if (nrec > 0 && !b->offsets) return false;
  return true;
}

// Backward workspace: per-pair gradients [capacity][9] floats, the per-record
// planes [kRecPlanes][round_up(V*n, 64)] floats, then one byte per pair (row
// written this step), padded so that whole words can be read past the end.
size_t grad_pair_bytes(uint64_t capacity) { return align256(sizeof(float) * GS_GRAD_FLOATS * (size_t)capacity); }
int64_t rec_stride(int64_t nrec) { return (nrec + 63) / 64 * 64; }
size_t rec_bytes(int64_t nrec) { return sizeof(float) * kRecPlanes * (size_t)rec_stride(nrec); }
size_t live_bytes(uint64_t capacity) { return align256((size_t)capacity + 256); }
size_t bwd_ws_bytes(uint64_t capacity, int64_t nrec) {
  return grad_pair_bytes(capacity) + rec_bytes(nrec) + live_bytes(capacity);
}
uint8_t* pair_live_ptr(const void* ws, uint64_t capacity, int64_t nrec) {
  return (uint8_t*)ws + grad_pair_bytes(capacity) + rec_bytes(nrec);
}

// Bytes the forward and backward need: the backward's regions, then the chunk states.
size_t render_ws_bytes(uint64_t capacity, int64_t nrec, const gs_opts* o) {
  return bwd_ws_bytes(capacity, nrec) + render_state_bytes(capacity, o);
}

// The fused forward + backward launch adds its tile flags, ticket and backward
// work list after the render regions.
size_t fused_ws_bytes(uint64_t capacity, int64_t nrec, const gs_opts* o, int64_t total_tiles) {
  return render_ws_bytes(capacity, nrec, o) +
         align256(4 * (size_t)fused_sync_words(total_tiles, chunk_slots(capacity, o)));
}
uint32_t* fused_sync_ptr(void* ws, uint64_t capacity, int64_t nrec, const gs_opts* o) {
  return (uint32_t*)((char*)ws + render_ws_bytes(capacity, nrec, o));
}

void attach_state(RenderArgs* a, uint64_t capacity, int64_t nrec, const gs_opts* o, const void* ws) {
  a->pair_live = pair_live_ptr(ws, capacity, nrec);
  char* base = (char*)ws + bwd_ws_bytes(capacity, nrec);
  a->slot_owner = (uint32_t*)base;
  a->state = (float4*)(base + state_owner_bytes(capacity, o));
  if (o->fwd_chunk) {
    char* f = base + state_owner_bytes(capacity, o) +
              align256(16 * (size_t)chunk_slots(capacity, o) * (size_t)(o->tile_w * o->tile_h));
    const FwdChunkWs w = fwd_chunk_ws(capacity, o);
    a->fslot_owner = (uint32_t*)(f + w.owner);
    a->fprod = (float*)(f + w.prod);
    a->fres = (float4*)(f + w.res);
    a->flast = (int32_t*)(f + w.last);
    a->fsuf = (float4*)(f + w.suf);
  }
}

ProjectBwdArgs project_bwd_args(ProjectArgs pa, const gs_opts* opts, const gs_projected* proj, const gs_binning* bins,
                                const float* grad_pair, const gs_grads* grads, int deg, void* ws, int64_t nrec) {
  pa.near_plane = opts->near_plane;
  pa.inv_tw = 1.0f / (float)opts->tile_w;
  pa.inv_th = 1.0f / (float)opts->tile_h;
  ProjectBwdArgs b;
  b.p = pa;
  b.grad_pair = grad_pair;
  b.rec = (float*)((char*)ws + grad_pair_bytes(bins->capacity));
  b.rec_stride = rec_stride(nrec);
  b.pair_live = pair_live_ptr(ws, bins->capacity, nrec);
  b.tiles_touched = proj->tiles_touched;
  b.offsets = bins->offsets;
  b.status = bins->status;
  b.g_means = grads->means;
  b.g_log_scales = grads->log_scales;
  b.g_quats = grads->quats;
  b.g_opacity_logits = grads->opacity_logits;
  b.g_sh_dc = grads->sh_dc;
  b.g_sh_rest = deg > 0 ? grads->sh_rest : nullptr;
  b.g_mask_logits = grads->mask_logits;
  b.g_sh_mask_logits = deg > 0 ? grads->sh_mask_logits : nullptr;
  b.assign = grads->assign != 0;
  b.g_mean2d = grads->mean2d;
  return b;
}

}  // namespace

extern "C" {

const char* gs_strerror(int code) {
  switch (code) {
    case GS_OK: return "ok";
    case GS_E_INVALID: return "invalid argument";
    case GS_E_CAPACITY: return "binning capacity exceeded";
    case GS_E_HIP: return "HIP launch failure";
    case GS_E_UNSUPPORTED: return "device is not gfx950";
    case GS_E_TOO_LARGE: return "input larger than the static scratch of the allocation-free entry point "
                                "(gs_mask_loss_noalloc: at most 2^24 Gaussians)";
    default: return "unknown error";
  }
}

int gs_view_sizes(const gs_camera* cams, int32_t V, const gs_opts* opts, int64_t* total_tiles,
                  int64_t* total_pixels) {
  ViewTable vt;
  int64_t px = 0;
  if (!view_table(cams, V, opts, &vt, &px)) return GS_E_INVALID;
  if (total_tiles) *total_tiles = vt.total_tiles;
  if (total_pixels) *total_pixels = px;
  return GS_OK;
}

size_t gs_workspace_size(int64_t n, int32_t V, const gs_camera* cams, const gs_opts* opts, uint64_t capacity) {
  ViewTable vt;
  if (n < 0 || capacity >= (1ull << 32) || !view_table(cams, V, opts, &vt, nullptr)) return 0;
  const SortPlan p = sort_plan(n, V, vt.total_tiles, capacity);
  const size_t sort_bytes = bin_sort_ws_bytes(p);
  const size_t render_bytes = fused_ws_bytes(capacity, (int64_t)V * n, opts, vt.total_tiles);
  return sort_bytes > render_bytes ? sort_bytes : render_bytes;
}

int gs_project(const gs_gaussians* g, const gs_camera* cams, int32_t V, const gs_opts* opts, gs_projected* out,
               gs_stream_t stream) {
  ProjectArgs a;
  ViewTable vt;
  if (!gaussians_ok(g, &a) || !view_table(cams, V, opts, &vt, nullptr)) return GS_E_INVALID;
  set_lowpass(&vt, opts, g->n);
  if (!out || (g->n > 0 && (!out->splats || !out->tiles_touched))) return GS_E_INVALID;
  if (((uintptr_t)out->splats & 15) != 0) return GS_E_INVALID;
  const int d = device_ok();
  if (d != GS_OK) return d;
  a.near_plane = opts->near_plane;
  a.inv_tw = 1.0f / (float)opts->tile_w;
  a.inv_th = 1.0f / (float)opts->tile_h;
  a.splats = (float4*)out->splats;
  a.tiles_touched = out->tiles_touched;
  return launched(launch_project(a, vt, g->sh_degree, (hipStream_t)stream));
}

int gs_bin_sort(const gs_projected* proj, const gs_camera* cams, int32_t V, int64_t n, const gs_opts* opts,
                gs_binning* out, void* ws, size_t ws_bytes, gs_stream_t stream) {
  ViewTable vt;
  if (!proj || n < 0 || n >= (1ll << 31) || !view_table(cams, V, opts, &vt, nullptr)) return GS_E_INVALID;
  if ((int64_t)V * n >= (1ll << 32)) return GS_E_INVALID;
  if (n > 0 && (!proj->splats || !proj->tiles_touched)) return GS_E_INVALID;
  if (!binning_ok(out, (int64_t)V * n)) return GS_E_INVALID;
  if (ws_bytes < gs_workspace_size(n, V, cams, opts, out->capacity) || (!ws && ws_bytes > 0) || !aligned(ws, 256))
    return GS_E_INVALID;
  const int d = device_ok();
  if (d != GS_OK) return d;
  const SortPlan p = sort_plan(n, V, vt.total_tiles, out->capacity);
  BinOut bo;
  bo.keys = out->keys;
  bo.ids = out->ids;
  bo.pair_index = out->pair_index;
  bo.offsets = out->offsets;
  bo.ranges = out->ranges;
  bo.order = out->order;
  bo.count = out->count;
  bo.status = out->status;
  return launched(launch_bin_sort(p, (const float4*)proj->splats, proj->tiles_touched, n, vt,
                                  1.0f / (float)opts->tile_w, 1.0f / (float)opts->tile_h, bo, out->capacity, ws,
                                  (hipStream_t)stream));
}

int gs_render_fwd(const gs_projected* proj, const gs_binning* bins, const gs_camera* cams, int32_t V, int64_t n,
                  const gs_opts* opts, float* image, float* T_final, int32_t* last_contrib, void* ws,
                  size_t ws_bytes, gs_stream_t stream) {
  ViewTable vt;
  if (!proj || n < 0 || !view_table(cams, V, opts, &vt, nullptr)) return GS_E_INVALID;
  if (!image || !T_final || !last_contrib || !binning_ok(bins, (int64_t)V * n)) return GS_E_INVALID;
  if (n > 0 && !proj->splats) return GS_E_INVALID;
  if (!ws || ws_bytes < render_ws_bytes(bins->capacity, (int64_t)V * n, opts) || !aligned(ws, 256))
    return GS_E_INVALID;
  const int d = device_ok();
  if (d != GS_OK) return d;
  RenderArgs a = render_args(proj, bins, opts);
  attach_state(&a, bins->capacity, (int64_t)V * n, opts, ws);
  return launched(launch_render_fwd(a, vt, image, T_final, last_contrib, (hipStream_t)stream));
}

int gs_render_bwd(const gs_gaussians* g, const gs_camera* cams, int32_t V, const gs_opts* opts,
                  const gs_projected* proj, const gs_binning* bins, const float* T_final,
                  const int32_t* last_contrib, const float* dL_dimage, gs_grads* grads, void* ws, size_t ws_bytes,
                  gs_stream_t stream) {
  ProjectArgs pa;
  ViewTable vt;
  if (!gaussians_ok(g, &pa) || !view_table(cams, V, opts, &vt, nullptr)) return GS_E_INVALID;
  set_lowpass(&vt, opts, g->n);
  if (!proj || !T_final || !last_contrib || !dL_dimage || !grads) return GS_E_INVALID;
  if (!binning_ok(bins, (int64_t)V * g->n)) return GS_E_INVALID;
  if (g->n > 0 && (!proj->splats || !proj->tiles_touched)) return GS_E_INVALID;
  const int64_t nrec = (int64_t)V * g->n;
  if (!ws || ws_bytes < render_ws_bytes(bins->capacity, nrec, opts) || !aligned(ws, 256)) return GS_E_INVALID;
  const int d = device_ok();
  if (d != GS_OK) return d;
  hipStream_t s = (hipStream_t)stream;
  float* grad_pair = (float*)ws;
  RenderArgs ra = render_args(proj, bins, opts);
  attach_state(&ra, bins->capacity, nrec, opts, ws);
  hipError_t e = launch_fill_u32((uint32_t*)ra.pair_live, (int64_t)(live_bytes(bins->capacity) / 4), 0u, s);
  if (e == hipSuccess) e = launch_render_bwd(ra, vt, T_final, last_contrib, dL_dimage, grad_pair, s);
  if (e != hipSuccess) return GS_E_HIP;
  return launched(launch_project_bwd(project_bwd_args(pa, opts, proj, bins, grad_pair, grads, g->sh_degree, ws, nrec),
                                     vt, g->sh_degree, s));
}

int gs_render_fwd_bwd_l2(const gs_gaussians* g, const gs_camera* cams, int32_t V, const gs_opts* opts,
                         const gs_projected* proj, const gs_binning* bins, const float* target, int32_t mean_views,
                         float* image, float* T_final, int32_t* last_contrib, float* dL_dimage, gs_grads* grads,
                         void* ws, size_t ws_bytes, gs_stream_t stream) {
  ProjectArgs pa;
  ViewTable vt;
  if (!gaussians_ok(g, &pa) || !view_table(cams, V, opts, &vt, nullptr)) return GS_E_INVALID;
  set_lowpass(&vt, opts, g->n);
  if (!proj || !target || mean_views < 1 || !image || !T_final || !last_contrib || !grads) return GS_E_INVALID;
  if (dL_dimage && (dL_dimage == image || dL_dimage == target)) return GS_E_INVALID;
  if (!binning_ok(bins, (int64_t)V * g->n)) return GS_E_INVALID;
  if (g->n > 0 && (!proj->splats || !proj->tiles_touched)) return GS_E_INVALID;
  const int64_t nrec = (int64_t)V * g->n;
  if (!ws || ws_bytes < fused_ws_bytes(bins->capacity, nrec, opts, vt.total_tiles) || !aligned(ws, 256))
    return GS_E_INVALID;
  float scale[GS_MAX_VIEWS];
  for (int v = 0; v < V; ++v)  // as gs_l2_grad: 2 / (3 H W mean_views)
    scale[v] = (float)(2.0 / ((double)(3 * (int64_t)cams[v].width * cams[v].height) * (double)mean_views));
  if (opts->fwd_chunk != 0) {  // forward chunking: the three separate calls
    if (!dL_dimage) return GS_E_INVALID;  // the separate backward reads dL/dimage from memory
    int r = gs_render_fwd(proj, bins, cams, V, g->n, opts, image, T_final, last_contrib, ws, ws_bytes, stream);
    if (r != GS_OK) return r;
    r = gs_l2_grad(image, target, cams, V, mean_views, dL_dimage, stream);
    if (r != GS_OK) return r;
    return gs_render_bwd(g, cams, V, opts, proj, bins, T_final, last_contrib, dL_dimage, grads, ws, ws_bytes,
                         stream);
  }
  const int d = device_ok();
  if (d != GS_OK) return d;
  hipStream_t s = (hipStream_t)stream;
  float* grad_pair = (float*)ws;
  RenderArgs ra = render_args(proj, bins, opts);
  attach_state(&ra, bins->capacity, nrec, opts, ws);
  hipError_t e = launch_fill_u32((uint32_t*)ra.pair_live, (int64_t)(live_bytes(bins->capacity) / 4), 0u, s);
  if (e == hipSuccess)
    e = launch_render_fused(ra, vt, image, T_final, last_contrib, target, scale, dL_dimage, grad_pair,
                            fused_sync_ptr(ws, bins->capacity, nrec, opts), s);
  if (e != hipSuccess) return GS_E_HIP;
  return launched(launch_project_bwd(project_bwd_args(pa, opts, proj, bins, grad_pair, grads, g->sh_degree, ws, nrec),
                                     vt, g->sh_degree, s));
}

int gs_count_hits(const gs_projected* proj, const gs_binning* bins, const gs_camera* cams, int32_t V, int64_t n,
                  const gs_opts* opts, uint32_t* hits, gs_stream_t stream) {
  ViewTable vt;
  if (!proj || n < 0 || !view_table(cams, V, opts, &vt, nullptr)) return GS_E_INVALID;
  if (!binning_ok(bins, (int64_t)V * n)) return GS_E_INVALID;
  if (n > 0 && (!proj->splats || !hits)) return GS_E_INVALID;
  const int d = device_ok();
  if (d != GS_OK) return d;
  RenderArgs a = render_args(proj, bins, opts);
  a.hits = hits;
  a.n = n;
  return launched(launch_count_hits(a, vt, (hipStream_t)stream));
}

size_t gs_significance_workspace_size(void) { return sizeof(SelectState); }

int gs_significance(const gs_gaussians* g, const uint32_t* hits, float volume_quantile, float* score, void* ws,
                    size_t ws_bytes, gs_stream_t stream) {
  if (!g || g->n < 0 || g->n >= (1ll << 32)) return GS_E_INVALID;
  if (!(volume_quantile > 0.0f && volume_quantile <= 1.0f)) return GS_E_INVALID;
  const int64_t n = g->n;
  if (n > 0 && (!g->log_scales || !g->opacity_logits || !hits || !score)) return GS_E_INVALID;
  if (!ws || ws_bytes < sizeof(SelectState)) return GS_E_INVALID;
  float thr = 0.0f;
  if (g->mask_logits && !mask_threshold(g->mask_eps, &thr)) return GS_E_INVALID;
  const int d = device_ok();
  if (d != GS_OK) return d;
  const int64_t r = std::min<int64_t>(std::max<int64_t>((int64_t)std::ceil((double)volume_quantile * (double)n), 1), n);
  return launched(launch_significance(g->log_scales, g->opacity_logits, g->mask_logits, thr, hits, n,
                                      (uint32_t)(r - 1), (SelectState*)ws, score, (hipStream_t)stream));
}

int gs_blend_bwd(const gs_camera* cams, int32_t V, int64_t n, const gs_opts* opts, const gs_projected* proj,
                 const gs_binning* bins, const float* T_final, const int32_t* last_contrib, const float* dL_dimage,
                 float* grad_pair, const void* ws, size_t ws_bytes, gs_stream_t stream) {
  ViewTable vt;
  if (n < 0 || !view_table(cams, V, opts, &vt, nullptr)) return GS_E_INVALID;
  if (!proj || !T_final || !last_contrib || !dL_dimage || !binning_ok(bins, (int64_t)V * n)) return GS_E_INVALID;
  if (n > 0 && (!proj->splats || !grad_pair || !aligned(grad_pair, 16))) return GS_E_INVALID;
  if (!ws || ws_bytes < render_ws_bytes(bins->capacity, (int64_t)V * n, opts) || !aligned(ws, 256))
    return GS_E_INVALID;
  const int d = device_ok();
  if (d != GS_OK) return d;
  RenderArgs ra = render_args(proj, bins, opts);
  attach_state(&ra, bins->capacity, (int64_t)V * n, opts, ws);
  const hipError_t e =
      launch_fill_u32((uint32_t*)ra.pair_live, (int64_t)(live_bytes(bins->capacity) / 4), 0u, (hipStream_t)stream);
  if (e != hipSuccess) return GS_E_HIP;
  return launched(launch_render_bwd(ra, vt, T_final, last_contrib, dL_dimage, grad_pair, (hipStream_t)stream));
}

int gs_project_bwd(const gs_gaussians* g, const gs_camera* cams, int32_t V, const gs_opts* opts,
                   const gs_projected* proj, const gs_binning* bins, const float* grad_pair, gs_grads* grads,
                   void* ws, size_t ws_bytes, gs_stream_t stream) {
  ProjectArgs pa;
  ViewTable vt;
  if (!gaussians_ok(g, &pa) || !view_table(cams, V, opts, &vt, nullptr)) return GS_E_INVALID;
  set_lowpass(&vt, opts, g->n);
  if (!proj || !grads || !binning_ok(bins, (int64_t)V * g->n)) return GS_E_INVALID;
  if (g->n > 0 && (!grad_pair || !proj->tiles_touched)) return GS_E_INVALID;
  const int64_t nrec = (int64_t)V * g->n;
  const size_t need = bwd_ws_bytes(bins->capacity, nrec);
  if (ws_bytes < need || (!ws && need > 0) || !aligned(ws, 256) || !aligned(grad_pair, 16)) return GS_E_INVALID;
  const int d = device_ok();
  if (d != GS_OK) return d;
  return launched(launch_project_bwd(project_bwd_args(pa, opts, proj, bins, grad_pair, grads, g->sh_degree, ws, nrec),
                                     vt, g->sh_degree, (hipStream_t)stream));
}

// ---------------------------------------------------------------------------
// Photometric loss (Eq. 7, L1 and D-SSIM terms)

static bool loss_views(const gs_camera* cams, int32_t V, int tile, LossViews* lv, int64_t* total_px) {
  if (!cams || V < 1 || V > GS_MAX_VIEWS) return false;
  std::memset(lv, 0, sizeof(*lv));
  int64_t po = 0, bo = 0;
  for (int v = 0; v < V; ++v) {
    const int W = cams[v].width, H = cams[v].height;
    if (W <= 0 || H <= 0) return false;
    LossView& q = lv->v[v];
    q.W = W, q.H = H;
    q.TX = (W + tile - 1) / tile, q.TY = (H + tile - 1) / tile;
    q.pix_off = po;
    q.block_off = (int32_t)bo;
    po += (int64_t)W * H;
    bo += 3ll * q.TX * q.TY;
    if (bo >= (1ll << 31)) return false;
  }
  lv->nviews = V;
  lv->total_blocks = (int32_t)bo;
  // the window's 1-D factor: exp(-k^2 / (2 * 1.5^2)), k = -5..5, normalised
  double g[11], sum = 0.0;
  for (int k = 0; k < 11; ++k) sum += (g[k] = std::exp(-(double)((k - 5) * (k - 5)) / (2.0 * 1.5 * 1.5)));
  for (int k = 0; k < 11; ++k) lv->g[k] = (float)(g[k] / sum);
  if (total_px) *total_px = po;
  return true;
}

struct LossWs {
  float* dmap;
  float* bsum;
  double* per_view;
  size_t bytes;
};

static LossWs loss_ws(const LossViews& lv, int64_t total_px, void* ws) {
  LossWs w{};
  char* b = (char*)ws;
  size_t o = 0;
  w.dmap = (float*)(b + o), o += align256(sizeof(float) * 9 * (size_t)total_px);
  w.bsum = (float*)(b + o), o += align256(sizeof(float) * 2 * (size_t)lv.total_blocks);
  w.per_view = (double*)(b + o), o += align256(sizeof(double) * GS_MAX_VIEWS);
  w.bytes = o;
  return w;
}

size_t gs_loss_workspace_size(const gs_camera* cams, int32_t V) {
  LossViews lv;
  int64_t px = 0;
  if (!loss_views(cams, V, kLossTile, &lv, &px)) return 0;
  return loss_ws(lv, px, nullptr).bytes;
}

int gs_loss_l1_dssim(const float* image, const float* target, const gs_camera* cams, int32_t V, float lambda_ssim,
                     float* loss, float* dL_dimage, void* ws, size_t ws_bytes, gs_stream_t stream) {
  LossViews lv;
  int64_t px = 0;
  if (!loss_views(cams, V, kLossTile, &lv, &px)) return GS_E_INVALID;
  if (!image || !target || !std::isfinite(lambda_ssim) || lambda_ssim < 0.0f || lambda_ssim > 1.0f)
    return GS_E_INVALID;
  const LossWs w = loss_ws(lv, px, ws);
  if (!ws || ws_bytes < w.bytes) return GS_E_INVALID;
  const int d = device_ok();
  if (d != GS_OK) return d;
  return launched(launch_loss(lv, image, target, lambda_ssim, loss, dL_dimage, w.dmap, w.bsum, w.per_view,
                              (hipStream_t)stream));
}

int gs_l2_grad(const float* image, const float* target, const gs_camera* cams, int32_t V, int32_t mean_views,
               float* dL_dimage, gs_stream_t stream) {
  if (!cams || V < 1 || V > GS_MAX_VIEWS || mean_views < 1 || !image || !target || !dL_dimage) return GS_E_INVALID;
  if (dL_dimage == image || dL_dimage == target) return GS_E_INVALID;
  L2Args a;
  a.nviews = V;
  int64_t end = 0;
  for (int v = 0; v < V; ++v) {
    if (cams[v].width <= 0 || cams[v].height <= 0) return GS_E_INVALID;
    const int64_t k = 3 * (int64_t)cams[v].width * cams[v].height;
    end += k;
    a.end[v] = end;
    a.scale[v] = (float)(2.0 / ((double)k * (double)mean_views));
  }
  if (end >= ((int64_t)1 << 31) * 256) return GS_E_INVALID;
  const int d = device_ok();
  if (d != GS_OK) return d;
  return launched(launch_l2_grad(image, target, dL_dimage, a, (hipStream_t)stream));
}

int gs_blur_views(const float* in, float* out, const gs_camera* cams, int32_t V, int32_t ksize, float sigma,
                  gs_stream_t stream) {
  BlurArgs b;
  int64_t px = 0;
  if (!loss_views(cams, V, kBlurTile, &b.views, &px)) return GS_E_INVALID;
  if (!in || !out || in == out) return GS_E_INVALID;
  if (ksize < 1 || ksize > 2 * kMaxBlurRadius + 1 || ksize % 2 == 0) return GS_E_INVALID;
  if (!std::isfinite(sigma) || !(sigma > 0.0f)) return GS_E_INVALID;
  const int d = device_ok();
  if (d != GS_OK) return d;
  b.r = (ksize - 1) / 2;
  double g[2 * kMaxBlurRadius + 1], sum = 0.0;
  for (int k = 0; k < ksize; ++k) {
    const double t = (double)(k - b.r);
    sum += (g[k] = std::exp(-t * t / (2.0 * (double)sigma * (double)sigma)));
  }
  for (int k = 0; k < 2 * kMaxBlurRadius + 1; ++k) b.g[k] = k < ksize ? (float)(g[k] / sum) : 0.0f;
  return launched(launch_blur(in, out, b, (hipStream_t)stream));
}

int gs_resize_views(const float* in, const gs_camera* in_cams, float* out, const gs_camera* out_cams, int32_t V,
                    gs_stream_t stream) {
  if (!in || !out || !in_cams || !out_cams || V < 1 || V > GS_MAX_VIEWS) return GS_E_INVALID;
  ResizeArgs a;
  std::memset(&a, 0, sizeof(a));
  int64_t io = 0, oo = 0;
  for (int v = 0; v < V; ++v) {
    ResizeView& q = a.v[v];
    q.W = in_cams[v].width, q.H = in_cams[v].height;
    q.Wo = out_cams[v].width, q.Ho = out_cams[v].height;
    if (q.W <= 0 || q.H <= 0 || q.Wo <= 0 || q.Ho <= 0) return GS_E_INVALID;
    q.in_off = io, q.out_off = oo;
    q.inv_area = (float)(1.0 / ((double)q.W * (double)q.H));
    io += (int64_t)q.W * q.H;
    oo += (int64_t)q.Wo * q.Ho;
    if (3 * io >= (1ll << 40) || 3 * oo >= (1ll << 40)) return GS_E_INVALID;
  }
  a.nviews = V;
  a.total_out = 3 * oo;
  // the buffers must not overlap: every output value reads other input values
  const char *i0 = (const char*)in, *i1 = i0 + 12 * io, *o0 = (const char*)out, *o1 = o0 + 12 * oo;
  if (i0 < o1 && o0 < i1) return GS_E_INVALID;
  const int d = device_ok();
  if (d != GS_OK) return d;
  return launched(launch_resize(in, out, a, (hipStream_t)stream));
}

size_t gs_mask_loss_workspace_size(int64_t n) {
  if (n < 0) return 0;
  return align256(sizeof(float) * 2 * (size_t)((n + 255) / 256)) + 256;
}

int gs_mask_loss(const gs_gaussians* g, float lambda_m, float lambda_sh, float* loss, gs_grads* grads, void* ws,
                 size_t ws_bytes, gs_stream_t stream) {
  if (!g || g->n < 0 || g->sh_degree < 0 || g->sh_degree > 3) return GS_E_INVALID;
  if (!std::isfinite(lambda_m) || !std::isfinite(lambda_sh)) return GS_E_INVALID;
  if (g->n > 0 && (!ws || ws_bytes < gs_mask_loss_workspace_size(g->n))) return GS_E_INVALID;
  const int d = device_ok();
  if (d != GS_OK) return d;
  float* gm = grads ? grads->mask_logits : nullptr;
  float* gsh = grads ? grads->sh_mask_logits : nullptr;
  return launched(launch_mask_loss(g->mask_logits, g->sh_mask_logits, g->n, g->sh_degree, lambda_m, lambda_sh, gm,
                                   gsh, loss, (float*)ws, (hipStream_t)stream));
}

int gs_mask_loss_noalloc(const gs_gaussians* g, float lambda_m, float lambda_sh, float* loss, gs_grads* grads,
                         gs_stream_t stream) {
  if (!g || g->n < 0 || g->sh_degree < 0 || g->sh_degree > 3) return GS_E_INVALID;
  if (!std::isfinite(lambda_m) || !std::isfinite(lambda_sh)) return GS_E_INVALID;
  if (g->n > kNoAllocMaxGaussians) return GS_E_TOO_LARGE;
  static_assert(2 * ((kNoAllocMaxGaussians + 255) / 256) <= (int64_t)kScratchFloats, "scratch too small");
  const int d = device_ok();
  if (d != GS_OK) return d;
  float* ws = scratch_on_current_device();
  if (!ws) return GS_E_HIP;
  float* gm = grads ? grads->mask_logits : nullptr;
  float* gsh = grads ? grads->sh_mask_logits : nullptr;
  // every partial sum the reduction reads is written first by the same call:
  // nothing in the scratch needs clearing
  return launched(launch_mask_loss(g->mask_logits, g->sh_mask_logits, g->n, g->sh_degree, lambda_m, lambda_sh, gm,
                                   gsh, loss, ws, (hipStream_t)stream));
}

}  // extern "C"
