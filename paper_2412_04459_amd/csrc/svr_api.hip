// Host side of the C ABI declared in include/svraster.h: argument checks,
// workspace layout, and the launch sequence of each stage.  No allocation
// happens here; every buffer is carved out of the caller's workspace.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <string>
#include <vector>

#include "svr_internal.h"

namespace svr {

// ---- kernel timing (diagnostics) -------------------------------------------
namespace {
std::mutex g_tmu;
bool g_timing = false;
std::vector<hipEvent_t> g_events;  // pool; pairs (start, stop)
size_t g_next = 0;
struct TimingRec {
  const char* name;
  int slot;
};
std::vector<TimingRec> g_recs;
constexpr size_t kEventPool = 16384;
}  // namespace

int timing_begin(hipStream_t s) {
  if (!g_timing) return -1;
  std::lock_guard<std::mutex> lk(g_tmu);
  if (g_next + 2 > g_events.size()) return -1;
  const int slot = (int)g_next;
  g_next += 2;
  if (hipEventRecord(g_events[slot], s) != hipSuccess) return -1;
  return slot;
}

void timing_end(int slot, const char* name, hipStream_t s) {
  if (slot < 0) return;
  std::lock_guard<std::mutex> lk(g_tmu);
  if (hipEventRecord(g_events[slot + 1], s) == hipSuccess) g_recs.push_back({name, slot});
}

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(SVR_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

#define SVR_HIP(call, what)                        \
  do {                                             \
    hipError_t e_ = (call);                        \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

int bits_for(int64_t x) {  // bits needed to hold values 0..x
  int b = 0;
  while (x > 0) {
    ++b;
    x >>= 1;
  }
  return b;
}

// Device camera records (fp64 centre, rotation, intrinsics, tile and pixel
// offsets of the concatenated images) for n_cams host cameras.
int fill_cams(const svr_camera* cams, int n_cams, int tile, CamSet* cs, int64_t* T_out,
              int64_t* P_out, int64_t* sat_out, int first_index = 0) {
  if (!cams) return fail(SVR_E_INVALID, "null camera pointer");
  if (n_cams < 1 || n_cams > SVR_MAX_CAMERAS)
    return fail(SVR_E_INVALID, "n_cams=%d outside 1..%d", n_cams, SVR_MAX_CAMERAS);
  const int tshift = tile == 8 ? 3 : (tile == 16 ? 4 : 5);
  int64_t T = 0, P = 0, sat = 0;
  cs->n = n_cams;
  cs->tile = tile;
  cs->tshift = tshift;
  for (int i = 0; i < n_cams; ++i) {
    const svr_camera& c = cams[i];
    if (c.width < 1 || c.height < 1 || c.width > 16384 || c.height > 16384)
      return fail(SVR_E_INVALID, "camera %d: size %dx%d outside 1..16384", first_index + i,
                  c.width, c.height);
    if (!(c.fx > 0.f) || !(c.fy > 0.f) || !isfinite(c.cx) || !isfinite(c.cy))
      return fail(SVR_E_INVALID, "camera %d: bad intrinsics", first_index + i);
    for (int k = 0; k < 12; ++k)
      if (!isfinite(c.w2c[k]))
        return fail(SVR_E_INVALID, "camera %d: non-finite pose", first_index + i);
    DevCam& d = cs->c[i];
    for (int r = 0; r < 3; ++r)
      for (int j = 0; j < 3; ++j) d.r[3 * r + j] = c.w2c[4 * r + j];
    for (int j = 0; j < 3; ++j) {
      double acc = 0;
      for (int r = 0; r < 3; ++r) acc += (double)c.w2c[4 * r + j] * (double)c.w2c[4 * r + 3];
      d.od[j] = -acc;
      d.o[j] = (float)(-acc);
    }
    d.fx = c.fx; d.fy = c.fy; d.cx = c.cx; d.cy = c.cy;
    d.W = c.width; d.H = c.height;
    d.ntx = (c.width + tile - 1) / tile;
    d.nty = (c.height + tile - 1) / tile;
    d.tile_off = (int32_t)T;
    d.sat_off = (int32_t)sat;
    d.pix_off = P;
    T += (int64_t)d.ntx * d.nty;
    sat += (int64_t)(d.ntx + 1) * (d.nty + 1);
    P += (int64_t)c.width * c.height;
  }
  *T_out = T;
  *P_out = P;
  *sat_out = sat;
  return SVR_OK;
}

int make_layout(const svr_scene* sc, const svr_camera* cams, int n_cams, const svr_opts* o,
                Layout* L, CamSet* cs) {
  if (!sc || !cams || !o || !L) return fail(SVR_E_INVALID, "null scene, camera or options pointer");
  if (n_cams < 1 || n_cams > SVR_MAX_CAMERAS)
    return fail(SVR_E_INVALID, "n_cams=%d outside 1..%d", n_cams, SVR_MAX_CAMERAS);
  if (sc->n_voxels < 0 || sc->n_voxels >= (int64_t)SVR_MAX_VOXELS)
    return fail(SVR_E_INVALID, "n_voxels=%lld outside [0, 2^29)", (long long)sc->n_voxels);
  if (sc->n_grid < 0) return fail(SVR_E_INVALID, "n_grid < 0");
  if (sc->sh_degree < 0 || sc->sh_degree > 3)
    return fail(SVR_E_INVALID, "sh_degree=%d outside 0..3", sc->sh_degree);
  if (sc->max_level < 1 || sc->max_level > SVR_MAX_LEVELS)
    return fail(SVR_E_INVALID, "max_level=%d outside 1..16", sc->max_level);
  if (sc->n_voxels > 0 && (!sc->center || !sc->size || !sc->octpath || !sc->vox_grid ||
                           !sc->grid_raw || !sc->sh))
    return fail(SVR_E_INVALID, "null scene array");
  if (o->K < 1 || o->K > SVR_MAX_K) return fail(SVR_E_INVALID, "K=%d outside 1..8", o->K);
  if (o->activation != SVR_ACT_EXPLIN && o->activation != SVR_ACT_SOFTPLUS)
    return fail(SVR_E_INVALID, "unknown activation %d", o->activation);
  if (!(o->t_stop >= 0.f && o->t_stop <= 1.f))
    return fail(SVR_E_INVALID, "t_stop outside [0, 1]");
  if (o->entry_capacity < 0 || o->entry_capacity >= (int64_t)1 << 30)
    return fail(SVR_E_INVALID, "entry_capacity outside [0, 2^30)");
  if (o->tile != 0 && o->tile != 8 && o->tile != 16 && o->tile != 32)
    return fail(SVR_E_INVALID, "tile=%d is not 8, 16 or 32", o->tile);
  if (o->persistent < 0) return fail(SVR_E_INVALID, "persistent < 0");
  if (o->accumulate != 0 && o->accumulate != 1) return fail(SVR_E_INVALID, "accumulate not 0/1");
  Layout& l = *L;
  memset(&l, 0, sizeof(l));
  memset(cs, 0, sizeof(*cs));
  l.N = sc->n_voxels;
  l.n_cams = n_cams;
  l.NV = l.N * n_cams;
  l.cap = o->entry_capacity;
  l.L = sc->max_level;
  l.tile = o->tile == 0 ? SVR_TILE : o->tile;
  l.tshift = l.tile == 8 ? 3 : (l.tile == 16 ? 4 : 5);
  l.persistent = o->persistent;
  int64_t T = 0, P = 0, sat = 0;
  int st = fill_cams(cams, n_cams, l.tile, cs, &T, &P, &sat);
  if (st != SVR_OK) return st;
  if (T >= ((int64_t)1 << 31)) return fail(SVR_E_INVALID, "too many tiles");
  l.T = (int32_t)T;
  l.P = P;
  l.sat_total = (int32_t)sat;
  cs->total_tiles = l.T;
  l.key_low = sc->order_rank ? bits_for(8 * l.N - 1) : 3 * l.L + 3;
  l.key_bits = bits_for(T - 1) + l.key_low;
  if (l.key_bits > 64)
    return fail(SVR_E_INVALID, "sort key needs %d bits (> 64): too many tiles for max_level %d",
                l.key_bits, l.L);
  // bucketing by tile: a counting sort (one scatter, result in the second
  // buffer) when the tile histogram fits in LDS and the keys are unique
  // within a tile (order ranks, or path keys of at most 15 levels), else
  // radix passes over the tile bits; the low key bits are sorted per tile
  l.count_sort = (T > 0 && T <= kCountTiles && (sc->order_rank != nullptr || l.L <= 15)) ? 1 : 0;
  l.passes = l.count_sort ? 1 : (l.key_bits - l.key_low + 7) / 8;
  l.scan_blocks = (l.NV + kBlock - 1) / kBlock;  // one partial per project/emit workgroup
  l.sort_parts = (l.cap + kSortPart - 1) / kSortPart;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t at_ = off;
    off = align_up(off + bytes, 256);
    return at_;
  };
  l.hdr = take(sizeof(WsHeader));
  l.count = take((size_t)l.NV * 4);
  l.rect = take((size_t)l.NV * 8);
  l.rec = take((size_t)l.NV * sizeof(VoxRec));
  l.scan_part = take((size_t)(l.scan_blocks > 0 ? l.scan_blocks : 1) * 8);
  l.tile_mask = take((size_t)T);
  l.tile_sat = take((size_t)sat * 4);
  // ranges, then the bucket counters and the chunk counter (cleared together)
  l.tile_range = take((size_t)T * 8 + (kOrderBuckets + 1) * 4);
  l.tile_order = take((size_t)T * 4);
  l.tile_rank = take((size_t)T * 4);
  l.tile_count = take((size_t)(l.count_sort ? T : 0) * 4);
  // a tile of n entries adds ceil(n / kBwdChunk) - 1 <= n / kBwdChunk chunks
  l.max_split = l.cap / kBwdChunk + 1;
  l.split_base = take((size_t)T * 4);
  l.split_items = take((size_t)l.max_split * 8);
  // items of the whole-grid emission pass (voxels of more than kBigEmit
  // entries or on tiles of several sign patterns, one item per kBigChunk
  // tiles); a frame with more emits the rest per thread
  l.max_big = l.cap / 16 + 1;
  l.big_list = take((size_t)l.max_big * 16);
  l.keys0 = take((size_t)l.cap * 8);
  l.keys1 = take((size_t)l.cap * 8);
  l.vals0 = take((size_t)l.cap * 4);
  l.vals1 = take((size_t)l.cap * 4);
  l.sort_hist = take(8 * 256 * 4);
  l.sort_status0 = take((size_t)(l.sort_parts > 0 ? l.sort_parts : 1) * 256 * 4);
  l.sort_status1 = take((size_t)(l.sort_parts > 0 ? l.sort_parts : 1) * 256 * 4);
  l.px_tau = take((size_t)P * 4);
  l.px_last = take((size_t)P * 4);
  l.ckpt = take((size_t)l.max_split * l.tile * l.tile * 16);
  l.ckpt_aux = take((size_t)l.max_split * l.tile * l.tile * 16);
  l.g_corner = take((size_t)l.N * 32);
  l.g_rgb = take((size_t)l.NV * 12);
  l.g_nrm = take((size_t)l.N * 12);
  l.total = off;
  return SVR_OK;
}

int check_ws(const Layout& L, void* ws, size_t ws_bytes) {
  if (!ws) return fail(SVR_E_INVALID, "null workspace");
  if ((reinterpret_cast<uintptr_t>(ws) & 255u) != 0)
    return fail(SVR_E_INVALID, "workspace must be 256-byte aligned");
  if (ws_bytes < L.total)
    return fail(SVR_E_WORKSPACE, "workspace has %zu bytes, %zu needed", ws_bytes, L.total);
  return SVR_OK;
}

const uint32_t* sorted_vals(const Layout& L, void* ws) {
  return at<uint32_t>(ws, (L.passes & 1) ? L.vals1 : L.vals0);
}
const uint64_t* sorted_keys(const Layout& L, void* ws) {
  return at<uint64_t>(ws, (L.passes & 1) ? L.keys1 : L.keys0);
}

}  // namespace
}  // namespace svr

using namespace svr;

extern "C" {

size_t svr_workspace_bytes(const svr_scene* scene, const svr_camera* cams, int n_cams,
                           const svr_opts* opts) {
  Layout L;
  CamSet cs;
  if (make_layout(scene, cams, n_cams, opts, &L, &cs) != SVR_OK) return 0;
  return L.total;
}

int svr_workspace_parts(const svr_scene* scene, const svr_camera* cams, int n_cams,
                        const svr_opts* opts, size_t* parts, int n_parts) {
  Layout L;
  CamSet cs;
  int st = make_layout(scene, cams, n_cams, opts, &L, &cs);
  if (st != SVR_OK) return st;
  if (!parts || n_parts < 0) return fail(SVR_E_INVALID, "null parts array");
  // region boundaries in layout order; each part is the span between them
  const size_t b[] = {L.hdr,       L.count,        L.scan_part,    L.tile_mask, L.keys0,
                      L.sort_hist, L.px_tau,       L.g_corner,     L.total};
  size_t v[SVR_WS_PARTS] = {0};
  v[0] = (b[1] - b[0]) + (b[4] - b[3]);  // header + tile tables
  v[1] = b[2] - b[1];                    // per (voxel, camera)
  v[2] = b[3] - b[2];                    // scan partials
  v[3] = b[5] - b[4];                    // keys + values, two buffers
  v[4] = b[6] - b[5];                    // sort histograms + status
  v[5] = b[7] - b[6];                    // per-pixel state
  v[6] = b[8] - b[7];                    // gradient scratch
  for (int i = 0; i < n_parts && i < SVR_WS_PARTS; ++i) parts[i] = v[i];
  return SVR_OK;
}

int svr_preprocess(const svr_scene* scene, const svr_camera* cams, int n_cams,
                   const svr_opts* opts, void* ws, size_t ws_bytes, int64_t* n_entries_out,
                   void* stream) {
  Layout L;
  CamSet cs;
  int st = make_layout(scene, cams, n_cams, opts, &L, &cs);
  if (st != SVR_OK) return st;
  if ((st = check_ws(L, ws, ws_bytes)) != SVR_OK) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  SVR_HIP(launch_tile_masks(cs, at<uint8_t>(ws, L.tile_mask), at<uint2>(ws, L.tile_range),
                            L.count_sort ? at<uint32_t>(ws, L.tile_count) : nullptr, s),
          "tile masks");
  SVR_HIP(launch_tile_sat(cs, at<uint8_t>(ws, L.tile_mask), at<uint32_t>(ws, L.tile_sat), s),
          "tile table");
  SVR_HIP(launch_project(*scene, cs, L, ws, s), "project");
  SVR_HIP(launch_scan(L, ws, s), "scan");
  if (n_entries_out) {
    unsigned long long E = 0;
    SVR_HIP(hipMemcpyAsync(&E, &at<WsHeader>(ws, L.hdr)->n_entries, sizeof(E),
                           hipMemcpyDeviceToHost, s),
            "read entry count");
    SVR_HIP(hipStreamSynchronize(s), "synchronise");
    *n_entries_out = (int64_t)E;
    if ((int64_t)E > L.cap)
      return fail(SVR_E_CAPACITY, "%llu entries exceed capacity %lld", E, (long long)L.cap);
  }
  SVR_HIP(launch_emit(*scene, cs, L, ws, s), "emit");
  return SVR_OK;
}

int svr_sort(const svr_scene* scene, const svr_camera* cams, int n_cams, const svr_opts* opts,
             void* ws, size_t ws_bytes, int64_t n_entries_hint, void* stream) {
  Layout L;
  CamSet cs;
  int st = make_layout(scene, cams, n_cams, opts, &L, &cs);
  if (st != SVR_OK) return st;
  if ((st = check_ws(L, ws, ws_bytes)) != SVR_OK) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int64_t n_max = (n_entries_hint >= 0 && n_entries_hint < L.cap) ? n_entries_hint : L.cap;
  WsHeader* hdr = at<WsHeader>(ws, L.hdr);
  // bucket by tile (the key bits above key_low), then sort each tile's range
  // by the low bits
  if (L.count_sort) {
    SVR_HIP(launch_tile_count_sort(L, ws, n_max, s), "tile counting sort");
  } else {
    bool in1 = false;
    SVR_HIP(launch_radix_sort(at<uint64_t>(ws, L.keys0), at<uint32_t>(ws, L.vals0),
                              at<uint64_t>(ws, L.keys1), at<uint32_t>(ws, L.vals1), &hdr->n_entries,
                              n_max, L.key_bits, L.key_low, at<uint32_t>(ws, L.sort_hist),
                              at<uint32_t>(ws, L.sort_status0), at<uint32_t>(ws, L.sort_status1),
                              hdr->tickets, &hdr->error, &in1, s),
            "radix sort");
    SVR_HIP(launch_tile_ranges(L, ws, sorted_keys(L, ws), s), "tile ranges");
  }
  const bool res1 = (L.passes & 1) != 0;
  SVR_HIP(launch_tile_sort(L, ws, res1 ? at<uint64_t>(ws, L.keys1) : at<uint64_t>(ws, L.keys0),
                           res1 ? at<uint32_t>(ws, L.vals1) : at<uint32_t>(ws, L.vals0),
                           res1 ? at<uint64_t>(ws, L.keys0) : at<uint64_t>(ws, L.keys1),
                           res1 ? at<uint32_t>(ws, L.vals0) : at<uint32_t>(ws, L.vals1), s),
          "tile sort");
  return SVR_OK;
}

int svr_render_fwd(const svr_scene* scene, const svr_camera* cams, int n_cams,
                   const svr_opts* opts, void* ws, size_t ws_bytes, float* rgba,
                   const svr_extra* extra, void* stream) {
  Layout L;
  CamSet cs;
  int st = make_layout(scene, cams, n_cams, opts, &L, &cs);
  if (st != SVR_OK) return st;
  if ((st = check_ws(L, ws, ws_bytes)) != SVR_OK) return st;
  if (!rgba && L.P > 0) return fail(SVR_E_INVALID, "null rgba");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  SVR_HIP(launch_render_fwd(*scene, cs, *opts, L, ws, sorted_vals(L, ws), rgba, extra, s),
          "render fwd");
  return SVR_OK;
}

int svr_render_bwd(const svr_scene* scene, const svr_camera* cams, int n_cams,
                   const svr_opts* opts, void* ws, size_t ws_bytes, const float* grad_rgba,
                   float* grad_grid, float* grad_sh, const svr_extra* extra,
                   void* stream) {
  Layout L;
  CamSet cs;
  int st = make_layout(scene, cams, n_cams, opts, &L, &cs);
  if (st != SVR_OK) return st;
  if ((st = check_ws(L, ws, ws_bytes)) != SVR_OK) return st;
  if (!grad_rgba && L.P > 0) return fail(SVR_E_INVALID, "null grad_rgba");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const bool aux = extra && (extra->grad_depth || extra->grad_normal);
  SVR_HIP(launch_render_bwd(*scene, cs, *opts, L, ws, sorted_vals(L, ws), grad_rgba, extra, s),
          "render bwd");
  SVR_HIP(launch_sh_bwd(*scene, cs, L, ws, grad_grid, grad_sh, opts->accumulate != 0, aux, s),
          "pre-process adjoint");
  return SVR_OK;
}

int svr_check_overflow(const svr_scene* scene, const svr_camera* cams, int n_cams,
                       const svr_opts* opts, void* ws, size_t ws_bytes,
                       int64_t* required_entries, void* stream) {
  Layout L;
  CamSet cs;
  int st = make_layout(scene, cams, n_cams, opts, &L, &cs);
  if (st != SVR_OK) return st;
  if ((st = check_ws(L, ws, ws_bytes)) != SVR_OK) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  WsHeader h;
  SVR_HIP(hipMemcpyAsync(&h, at<WsHeader>(ws, L.hdr), sizeof(h), hipMemcpyDeviceToHost, s),
          "read header");
  SVR_HIP(hipStreamSynchronize(s), "synchronise");
  if (required_entries) *required_entries = (int64_t)h.n_entries;
  if (h.error & 1u) return fail(SVR_E_DEVICE, "sort look-back exceeded its spin limit");
  if (h.error & 2u) return fail(SVR_E_DEVICE, "backward chunk list overflow");
  if (h.error & 4u)
    return fail(SVR_E_DEVICE, "tile counts disagree with the entry count (sort without its pre-process)");
  if ((int64_t)h.n_entries > L.cap)
    return fail(SVR_E_CAPACITY, "%llu entries exceed capacity %lld", h.n_entries,
                (long long)L.cap);
  return SVR_OK;
}

int svr_copy_sorted(const svr_scene* scene, const svr_camera* cams, int n_cams,
                    const svr_opts* opts, void* ws, size_t ws_bytes, uint64_t* keys,
                    uint32_t* values, int64_t n, void* stream) {
  Layout L;
  CamSet cs;
  int st = make_layout(scene, cams, n_cams, opts, &L, &cs);
  if (st != SVR_OK) return st;
  if ((st = check_ws(L, ws, ws_bytes)) != SVR_OK) return st;
  if (n < 0 || n > L.cap) return fail(SVR_E_INVALID, "n outside [0, capacity]");
  if (n == 0) return SVR_OK;
  if (!keys || !values) return fail(SVR_E_INVALID, "null output");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  SVR_HIP(hipMemcpyAsync(keys, sorted_keys(L, ws), (size_t)n * 8, hipMemcpyDeviceToDevice, s),
          "copy keys");
  SVR_HIP(hipMemcpyAsync(values, sorted_vals(L, ws), (size_t)n * 4, hipMemcpyDeviceToDevice, s),
          "copy values");
  return SVR_OK;
}

size_t svr_radix_sort_scratch_bytes(int64_t n, int bits) {
  if (n < 0 || bits < 0 || bits > 64) return 0;
  return align_up(sort_scratch_bytes(n, bits, nullptr), 256) + 256;
}

int svr_radix_sort_pairs(uint64_t* keys, uint32_t* values, uint64_t* keys_tmp,
                         uint32_t* values_tmp, int64_t n, int bits, void* scratch,
                         size_t scratch_bytes, void* stream) {
  if (n < 0 || n >= ((int64_t)1 << 30)) return fail(SVR_E_INVALID, "n outside [0, 2^30)");
  if (bits < 0 || bits > 64) return fail(SVR_E_INVALID, "bits outside 0..64");
  if (n == 0) return SVR_OK;
  if (!keys || !values || !keys_tmp || !values_tmp || !scratch)
    return fail(SVR_E_INVALID, "null pointer");
  if ((reinterpret_cast<uintptr_t>(scratch) & 255u) != 0)
    return fail(SVR_E_INVALID, "scratch must be 256-byte aligned");
  const size_t need = svr_radix_sort_scratch_bytes(n, bits);
  if (scratch_bytes < need)
    return fail(SVR_E_WORKSPACE, "scratch has %zu bytes, %zu needed", scratch_bytes, need);
  int64_t parts = 0;
  sort_scratch_bytes(n, bits, &parts);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  // [n as u64 | tickets 16 | err | pad] [hist 2048] [status0] [status1]
  uint32_t* base = reinterpret_cast<uint32_t*>(scratch);
  auto* n_dev = reinterpret_cast<unsigned long long*>(base);
  uint32_t* tickets = base + 2;
  uint32_t* err = base + 18;
  uint32_t* hist = base + 64;
  uint32_t* st0 = hist + 8 * 256;
  uint32_t* st1 = st0 + (parts > 0 ? parts : 1) * 256;
  SVR_HIP(launch_fill_u32(base, 0u, 64, s), "clear scratch");
  SVR_HIP(launch_fill_u32(base, (uint32_t)(n & 0xffffffffu), 1, s), "store n");
  bool in1 = false;
  SVR_HIP(launch_radix_sort(keys, values, keys_tmp, values_tmp, n_dev, n, bits, 0, hist, st0, st1,
                            tickets, err, &in1, s),
          "radix sort");
  if (in1) {
    SVR_HIP(hipMemcpyAsync(keys, keys_tmp, (size_t)n * 8, hipMemcpyDeviceToDevice, s), "copy keys");
    SVR_HIP(hipMemcpyAsync(values, values_tmp, (size_t)n * 4, hipMemcpyDeviceToDevice, s),
            "copy values");
  }
  return SVR_OK;
}

}  // extern "C"

// ---- the sort with library-held scratch --------------------------------------
// Layout of the array: [sort counters, histograms, status] [keys_tmp] [values_tmp],
// each part sized for SVR_STATIC_SORT_MAX pairs.
namespace svr {
namespace {
constexpr int64_t kStaticParts = (SVR_STATIC_SORT_MAX + kSortPart - 1) / kSortPart;
constexpr size_t kStaticHead =
    ((size_t)(8 * 256 + 2 * kStaticParts * 256 + 64) * 4 + 256 + 255) / 256 * 256;
constexpr size_t kStaticKeys = kStaticHead;
constexpr size_t kStaticVals = kStaticKeys + (size_t)SVR_STATIC_SORT_MAX * 8;
constexpr size_t kStaticEnd = kStaticVals + (size_t)SVR_STATIC_SORT_MAX * 4;
static_assert(kStaticEnd == SVR_STATIC_SORT_BYTES, "SVR_STATIC_SORT_BYTES is the array size");
constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
void* g_static_ptr[kMaxDevices] = {};
}  // namespace
}  // namespace svr

static __device__ __align__(256) unsigned char scratch[svr::kStaticEnd];

namespace svr {
namespace {
// Device address of `scratch` on the current device, looked up once per
// device (each GPU holds its own copy of the array at its own address).
int static_scratch(unsigned char** out) {
  int dev = -1;
  SVR_HIP(hipGetDevice(&dev), "current device");
  if (dev < 0 || dev >= kMaxDevices) return fail(SVR_E_INVALID, "device %d outside 0..63", dev);
  std::lock_guard<std::mutex> lk(g_static_mu);
  if (!g_static_ptr[dev]) {
    void* p = nullptr;
    SVR_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "address of the sort scratch array");
    if (!p) return fail(SVR_E_HIP, "null address of the sort scratch array");
    g_static_ptr[dev] = p;
  }
  *out = static_cast<unsigned char*>(g_static_ptr[dev]);
  return SVR_OK;
}
}  // namespace
}  // namespace svr

extern "C" {

int svr_radix_sort_pairs_static(uint64_t* keys, uint32_t* values, int64_t n, int bits,
                                void* stream) {
  if (n < 0 || n > (int64_t)SVR_STATIC_SORT_MAX)
    return fail(SVR_E_INVALID, "n=%lld outside [0, %d] (the library-held sort scratch)",
                (long long)n, SVR_STATIC_SORT_MAX);
  if (bits < 0 || bits > 64) return fail(SVR_E_INVALID, "bits outside 0..64");
  if (n == 0) return SVR_OK;
  if (!keys || !values) return fail(SVR_E_INVALID, "null pointer");
  int64_t parts = 0;
  if (align_up(sort_scratch_bytes(n, bits, &parts), 256) > kStaticHead)
    return fail(SVR_E_INVALID, "sort scratch exceeds the library-held array");
  unsigned char* ptr = nullptr;
  int st = static_scratch(&ptr);
  if (st != SVR_OK) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  // [n as u64 | tickets 16 | err | pad] [hist 2048] [status0] [status1], as in
  // svr_radix_sort_pairs
  uint32_t* base = reinterpret_cast<uint32_t*>(ptr);
  auto* n_dev = reinterpret_cast<unsigned long long*>(base);
  uint32_t* tickets = base + 2;
  uint32_t* err = base + 18;
  uint32_t* hist = base + 64;
  uint32_t* st0 = hist + 8 * 256;
  uint32_t* st1 = st0 + parts * 256;
  uint64_t* keys_tmp = reinterpret_cast<uint64_t*>(ptr + kStaticKeys);
  uint32_t* values_tmp = reinterpret_cast<uint32_t*>(ptr + kStaticVals);
  SVR_HIP(launch_fill_u32(base, 0u, 64, s), "clear scratch");
  SVR_HIP(launch_fill_u32(base, (uint32_t)(n & 0xffffffffu), 1, s), "store n");
  bool in1 = false;
  SVR_HIP(launch_radix_sort(keys, values, keys_tmp, values_tmp, n_dev, n, bits, 0, hist, st0, st1,
                            tickets, err, &in1, s),
          "radix sort");
  if (in1) {
    SVR_HIP(hipMemcpyAsync(keys, keys_tmp, (size_t)n * 8, hipMemcpyDeviceToDevice, s), "copy keys");
    SVR_HIP(hipMemcpyAsync(values, values_tmp, (size_t)n * 4, hipMemcpyDeviceToDevice, s),
            "copy values");
  }
  return SVR_OK;
}

int svr_atomic_probe(float* corner, float* colour, int64_t n_rows, int64_t n_waves, int iters,
                     void* stream) {
  if (!corner || !colour) return fail(SVR_E_INVALID, "null pointer");
  if (n_rows < 1 || n_rows >= ((int64_t)1 << 32)) return fail(SVR_E_INVALID, "n_rows outside [1, 2^32)");
  if (n_waves < 1 || n_waves > ((int64_t)1 << 26)) return fail(SVR_E_INVALID, "n_waves outside [1, 2^26]");
  if (iters < 0) return fail(SVR_E_INVALID, "iters < 0");
  if (iters == 0) return SVR_OK;
  SVR_HIP(launch_atomic_probe(corner, colour, n_rows, n_waves, iters,
                              reinterpret_cast<hipStream_t>(stream)),
          "atomic probe");
  return SVR_OK;
}

int svr_render_stats(const svr_scene* scene, const svr_camera* cams, int n_cams,
                     const svr_opts* opts, void* ws, size_t ws_bytes, int64_t* counts,
                     void* stream) {
  Layout L;
  CamSet cs;
  int st = make_layout(scene, cams, n_cams, opts, &L, &cs);
  if (st != SVR_OK) return st;
  if ((st = check_ws(L, ws, ws_bytes)) != SVR_OK) return st;
  if (!counts) return fail(SVR_E_INVALID, "null counts");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  SVR_HIP(launch_render_stats(*scene, cs, *opts, L, ws, sorted_vals(L, ws), s), "render stats");
  SVR_HIP(launch_count_inview(L, ws, s), "in-view count");
  WsHeader h;
  SVR_HIP(hipMemcpyAsync(&h, at<WsHeader>(ws, L.hdr), sizeof(h), hipMemcpyDeviceToHost, s),
          "read header");
  SVR_HIP(hipStreamSynchronize(s), "synchronise");
  counts[0] = (int64_t)(h.n_entries < (unsigned long long)L.cap ? h.n_entries : L.cap);
  counts[1] = (int64_t)h.stats[0];
  counts[2] = (int64_t)h.stats[1];
  counts[3] = (int64_t)h.stats[2];
  counts[4] = (int64_t)h.stats[3];
  return SVR_OK;
}

int svr_timing_enable(int on) {
  std::lock_guard<std::mutex> lk(g_tmu);
  if (on && g_events.empty()) {
    g_events.resize(kEventPool);
    for (size_t i = 0; i < kEventPool; ++i) {
      hipError_t e = hipEventCreate(&g_events[i]);
      if (e != hipSuccess) {
        g_events.resize(i);
        return hip_fail(e, "create timing events");
      }
    }
  }
  g_timing = on != 0;
  g_next = 0;
  g_recs.clear();
  return SVR_OK;
}

int svr_timing_read(char* names, int name_len, double* total_ms, int64_t* launches, int max_n,
                    int* n_out) {
  std::lock_guard<std::mutex> lk(g_tmu);
  if (!n_out || (max_n > 0 && (!names || !total_ms || !launches)) || name_len < 2)
    return fail(SVR_E_INVALID, "bad timing output arguments");
  int n = 0;
  std::vector<std::string> keys;
  std::vector<double> ms;
  std::vector<int64_t> cnt;
  for (const TimingRec& r : g_recs) {
    SVR_HIP(hipEventSynchronize(g_events[r.slot + 1]), "wait for timing event");
    float t = 0.f;
    SVR_HIP(hipEventElapsedTime(&t, g_events[r.slot], g_events[r.slot + 1]), "elapsed time");
    size_t k = 0;
    while (k < keys.size() && keys[k] != r.name) ++k;
    if (k == keys.size()) {
      keys.push_back(r.name);
      ms.push_back(0.0);
      cnt.push_back(0);
    }
    ms[k] += t;
    cnt[k] += 1;
  }
  for (size_t k = 0; k < keys.size() && n < max_n; ++k, ++n) {
    snprintf(names + (size_t)n * name_len, (size_t)name_len, "%s", keys[k].c_str());
    total_ms[n] = ms[k];
    launches[n] = cnt[k];
  }
  *n_out = n;
  g_next = 0;
  g_recs.clear();
  return SVR_OK;
}

namespace {
struct SvrGraph {
  hipGraph_t graph;
  hipGraphExec_t exec;
};
}  // namespace

int svr_graph_capture(const svr_scene* scene, const svr_camera* cams, int n_cams,
                      const svr_opts* opts, void* ws, size_t ws_bytes, float* rgba,
                      const float* grad_rgba, float* grad_grid, float* grad_sh,
                      const svr_extra* extra, void* stream, void** graph_out) {
  if (!graph_out) return fail(SVR_E_INVALID, "null graph_out");
  *graph_out = nullptr;
  if (!stream) return fail(SVR_E_INVALID, "capture needs a non-default stream");
  Layout L;
  CamSet cs;
  int st = make_layout(scene, cams, n_cams, opts, &L, &cs);
  if (st != SVR_OK) return st;
  if ((st = check_ws(L, ws, ws_bytes)) != SVR_OK) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  bool timing;
  {
    std::lock_guard<std::mutex> lk(g_tmu);
    timing = g_timing;
    g_timing = false;
  }
  SVR_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "begin capture");
  st = svr_preprocess(scene, cams, n_cams, opts, ws, ws_bytes, nullptr, stream);
  if (st == SVR_OK) st = svr_sort(scene, cams, n_cams, opts, ws, ws_bytes, -1, stream);
  if (st == SVR_OK)
    st = svr_render_fwd(scene, cams, n_cams, opts, ws, ws_bytes, rgba, extra, stream);
  if (st == SVR_OK && grad_rgba)
    st = svr_render_bwd(scene, cams, n_cams, opts, ws, ws_bytes, grad_rgba, grad_grid, grad_sh,
                        extra, stream);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(s, &g);
  {
    std::lock_guard<std::mutex> lk(g_tmu);
    g_timing = timing;
  }
  if (st != SVR_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess) return hip_fail(e, "end capture");
  hipGraphExec_t x = nullptr;
  e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    return hip_fail(e, "instantiate graph");
  }
  *graph_out = new SvrGraph{g, x};
  return SVR_OK;
}

int svr_graph_launch(void* graph, void* stream) {
  if (!graph) return fail(SVR_E_INVALID, "null graph");
  SvrGraph* G = static_cast<SvrGraph*>(graph);
  SVR_HIP(hipGraphLaunch(G->exec, reinterpret_cast<hipStream_t>(stream)), "graph launch");
  return SVR_OK;
}

int svr_graph_destroy(void* graph) {
  if (!graph) return SVR_OK;
  SvrGraph* G = static_cast<SvrGraph*>(graph);
  hipError_t e1 = hipGraphExecDestroy(G->exec);
  hipError_t e2 = hipGraphDestroy(G->graph);
  delete G;
  if (e1 != hipSuccess) return hip_fail(e1, "destroy graph exec");
  if (e2 != hipSuccess) return hip_fail(e2, "destroy graph");
  return SVR_OK;
}

size_t svr_grid_adjacency_scratch_bytes(int64_t n_voxels, int64_t n_grid) {
  if (n_voxels < 0 || n_voxels >= (int64_t)SVR_MAX_VOXELS || n_grid < 0 || n_grid >= ((int64_t)1 << 31))
    return 0;
  return grid_adjacency_scratch_bytes(n_voxels, n_grid) + 256;
}

size_t svr_order_rank_scratch_bytes(int64_t n_voxels, int max_level) {
  if (n_voxels < 0 || n_voxels >= (int64_t)SVR_MAX_VOXELS || max_level < 1 ||
      max_level > SVR_MAX_LEVELS)
    return 0;
  return order_rank_scratch_bytes(n_voxels, max_level) + 256;
}

int svr_build_order_ranks(const uint64_t* octpath, int64_t n_voxels, int max_level,
                          uint32_t* rank, void* scratch, size_t scratch_bytes, void* stream) {
  if (n_voxels < 0 || n_voxels >= (int64_t)SVR_MAX_VOXELS)
    return fail(SVR_E_INVALID, "n_voxels outside [0, 2^29)");
  if (max_level < 1 || max_level > SVR_MAX_LEVELS)
    return fail(SVR_E_INVALID, "max_level=%d outside 1..16", max_level);
  if (n_voxels > 0 && (!octpath || !rank || !scratch)) return fail(SVR_E_INVALID, "null pointer");
  if ((reinterpret_cast<uintptr_t>(scratch) & 255u) != 0)
    return fail(SVR_E_INVALID, "scratch must be 256-byte aligned");
  const size_t need = svr_order_rank_scratch_bytes(n_voxels, max_level);
  if (scratch_bytes < need)
    return fail(SVR_E_WORKSPACE, "scratch has %zu bytes, %zu needed", scratch_bytes, need);
  if (n_voxels == 0) return SVR_OK;
  SVR_HIP(launch_order_ranks(octpath, n_voxels, max_level, rank, scratch,
                             reinterpret_cast<hipStream_t>(stream)),
          "order ranks");
  return SVR_OK;
}

int svr_build_grid_adjacency(const int32_t* vox_grid, int64_t n_voxels, int64_t n_grid,
                             int32_t* adj_off, int32_t* adj, void* scratch, size_t scratch_bytes,
                             void* stream) {
  if (n_voxels < 0 || n_voxels >= (int64_t)SVR_MAX_VOXELS)
    return fail(SVR_E_INVALID, "n_voxels outside [0, 2^29)");
  if (n_grid < 0 || n_grid >= ((int64_t)1 << 31)) return fail(SVR_E_INVALID, "n_grid out of range");
  if (!adj_off || (n_voxels > 0 && (!vox_grid || !adj || !scratch)))
    return fail(SVR_E_INVALID, "null pointer");
  if ((reinterpret_cast<uintptr_t>(scratch) & 255u) != 0)
    return fail(SVR_E_INVALID, "scratch must be 256-byte aligned");
  const size_t need = svr_grid_adjacency_scratch_bytes(n_voxels, n_grid);
  if (scratch_bytes < need)
    return fail(SVR_E_WORKSPACE, "scratch has %zu bytes, %zu needed", scratch_bytes, need);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (n_voxels == 0) {
    SVR_HIP(launch_fill_u32(reinterpret_cast<uint32_t*>(adj_off), 0u, n_grid + 1, s), "clear offsets");
    return SVR_OK;
  }
  SVR_HIP(launch_grid_adjacency(vox_grid, n_voxels, n_grid, adj_off, adj, scratch, s),
          "grid adjacency");
  return SVR_OK;
}

int svr_downsample(const float* in, int w_in, int h_in, float* out, int w_out, int h_out,
                   const float* bg, void* stream) {
  if (w_out < 1 || h_out < 1 || w_in < w_out || h_in < h_out || w_in > 65536 || h_in > 65536)
    return fail(SVR_E_INVALID, "sizes %dx%d -> %dx%d: need 1 <= out <= in <= 65536", w_in, h_in,
                w_out, h_out);
  if (!in || !out) return fail(SVR_E_INVALID, "null image");
  const float zero[3] = {0.f, 0.f, 0.f};
  SVR_HIP(launch_downsample(in, w_in, h_in, out, w_out, h_out, bg ? bg : zero,
                            reinterpret_cast<hipStream_t>(stream)),
          "downsample");
  return SVR_OK;
}

int svr_downsample_bwd(const float* grad_out, int w_out, int h_out, float* grad_in, int w_in,
                       int h_in, const float* bg, void* stream) {
  if (w_out < 1 || h_out < 1 || w_in < w_out || h_in < h_out || w_in > 65536 || h_in > 65536)
    return fail(SVR_E_INVALID, "sizes %dx%d -> %dx%d: need 1 <= out <= in <= 65536", w_in, h_in,
                w_out, h_out);
  if (!grad_out || !grad_in) return fail(SVR_E_INVALID, "null image");
  const float zero[3] = {0.f, 0.f, 0.f};
  SVR_HIP(launch_downsample_bwd(grad_out, w_out, h_out, grad_in, w_in, h_in, bg ? bg : zero,
                                reinterpret_cast<hipStream_t>(stream)),
          "downsample adjoint");
  return SVR_OK;
}

// Image bytes per TSDF fusion launch (the MALL holds 256 MB).
constexpr int64_t kFuseGroupBytes = (int64_t)96 << 20;

int svr_tsdf_fuse(const float* grid_pos, int64_t n_grid, const svr_camera* cams, int n_cams,
                  const float* depth, const float* rgba, float min_alpha, float trunc, float* tsdf,
                  float* weight, const uint32_t* order, void* stream) {
  if (n_grid < 0 || n_grid >= ((int64_t)1 << 31))
    return fail(SVR_E_INVALID, "n_grid=%lld outside [0, 2^31)", (long long)n_grid);
  if (!(trunc > 0.f) || !isfinite(trunc)) return fail(SVR_E_INVALID, "trunc must be finite and > 0");
  if (!isfinite(min_alpha)) return fail(SVR_E_INVALID, "min_alpha must be finite");
  if (!cams || n_cams < 1) return fail(SVR_E_INVALID, "need at least one camera");
  // consecutive cameras in groups of at most SVR_MAX_CAMERAS whose images
  // (depth, plus rgba when given) stay within kFuseGroupBytes, one launch
  // each, so that a launch's pixel gathers stay resident in the caches; the
  // images stay one concatenated array
  std::vector<FuseCamSet> groups;
  int64_t pix_base = 0;
  for (int c0 = 0; c0 < n_cams;) {
    int nc = 0;
    int64_t bytes = 0;
    while (c0 + nc < n_cams && nc < SVR_MAX_CAMERAS) {
      const int64_t b = (int64_t)cams[c0 + nc].width * cams[c0 + nc].height * (rgba ? 20 : 4);
      // a Morton visit order keeps the gathers local at any footprint; it makes
      // the running sums' round trips between launches scattered instead
      if (nc > 0 && !order && bytes + b > kFuseGroupBytes) break;
      bytes += b;
      ++nc;
    }
    CamSet cs;  // validation, centres and pixel offsets
    memset(&cs, 0, sizeof(cs));
    int64_t T = 0, P = 0, sat = 0;
    int st = fill_cams(cams + c0, nc, SVR_TILE, &cs, &T, &P, &sat, c0);
    if (st != SVR_OK) return st;
    groups.emplace_back();
    FuseCamSet& fs = groups.back();
    memset(&fs, 0, sizeof(fs));
    fs.n = nc;
    for (int i = 0; i < nc; ++i) {
      const svr_camera& c = cams[c0 + i];
      FuseCam& f = fs.c[i];
      for (int j = 0; j < 3; ++j) f.od[j] = cs.c[i].od[j];
      for (int r = 0; r < 3; ++r) {
        for (int j = 0; j < 3; ++j) f.r[3 * r + j] = c.w2c[4 * r + j];
        f.t[r] = c.w2c[4 * r + 3];
      }
      f.fx = c.fx; f.fy = c.fy; f.cx = c.cx; f.cy = c.cy;
      f.W = c.width; f.H = c.height;
      f.pix_off = pix_base + cs.c[i].pix_off;
    }
    pix_base += P;
    c0 += nc;
  }
  const int n_groups = (int)groups.size();
  if (n_grid == 0) return SVR_OK;
  if (!grid_pos || !depth || !tsdf || !weight) return fail(SVR_E_INVALID, "null array");
  for (int gi = 0; gi < n_groups; ++gi)
    SVR_HIP(launch_tsdf_fuse(grid_pos, n_grid, groups[(size_t)gi], depth, rgba, min_alpha, trunc,
                             tsdf, weight, order, gi == 0, gi == n_groups - 1,
                             reinterpret_cast<hipStream_t>(stream)),
            "tsdf fusion");
  return SVR_OK;
}

int svr_mesh_case_table(uint8_t* counts, uint8_t* verts) {
  if (!counts || !verts) return fail(SVR_E_INVALID, "null table array");
  mesh_case_table(counts, verts);
  return SVR_OK;
}

int svr_marching_cubes(const svr_scene* scene, const float* field, const float* weight, float iso,
                       int64_t max_triangles, int32_t* tri_keys, float* tri_pos,
                       unsigned long long* n_triangles, const uint32_t* order, void* stream) {
  if (!scene) return fail(SVR_E_INVALID, "null scene");
  if (scene->n_voxels < 0 || scene->n_voxels >= (int64_t)SVR_MAX_VOXELS)
    return fail(SVR_E_INVALID, "n_voxels=%lld outside [0, 2^29)", (long long)scene->n_voxels);
  if (scene->n_grid < 0 || scene->n_grid >= ((int64_t)1 << 31))
    return fail(SVR_E_INVALID, "n_grid=%lld outside [0, 2^31)", (long long)scene->n_grid);
  if (!isfinite(iso)) return fail(SVR_E_INVALID, "iso must be finite");
  if (max_triangles < 0) return fail(SVR_E_INVALID, "max_triangles < 0");
  if (!n_triangles) return fail(SVR_E_INVALID, "null triangle counter");
  if (max_triangles > 0 && (!tri_keys || !tri_pos)) return fail(SVR_E_INVALID, "null triangle arrays");
  if (scene->n_voxels > 0 && (!scene->center || !scene->size || !scene->vox_grid || !field))
    return fail(SVR_E_INVALID, "null scene array or field");
  SVR_HIP(launch_mesh_cells(*scene, field, weight, iso, max_triangles, tri_keys, tri_pos,
                            n_triangles, order, reinterpret_cast<hipStream_t>(stream)),
          "marching cubes");
  return SVR_OK;
}

int svr_morton_keys(const float* pos, int64_t n, const float* lo, float extent, uint64_t* keys,
                    uint32_t* values, void* stream) {
  if (n < 0 || n >= ((int64_t)1 << 32)) return fail(SVR_E_INVALID, "n outside [0, 2^32)");
  if (!lo || !isfinite(lo[0]) || !isfinite(lo[1]) || !isfinite(lo[2]))
    return fail(SVR_E_INVALID, "lo must be 3 finite floats");
  if (!(extent > 0.f) || !isfinite(extent)) return fail(SVR_E_INVALID, "extent must be finite > 0");
  if (n == 0) return SVR_OK;
  if (!pos || !keys || !values) return fail(SVR_E_INVALID, "null array");
  SVR_HIP(launch_morton_keys(pos, n, lo, extent, keys, values, reinterpret_cast<hipStream_t>(stream)),
          "morton keys");
  return SVR_OK;
}

const char* svr_status_string(int status) {
  switch (status) {
    case SVR_OK: return "ok";
    case SVR_E_INVALID: return "invalid argument";
    case SVR_E_CAPACITY: return "entry capacity exceeded";
    case SVR_E_HIP: return "HIP runtime error";
    case SVR_E_WORKSPACE: return "workspace too small";
    case SVR_E_DEVICE: return "device-side failure";
    default: return "unknown status";
  }
}

const char* svr_last_error(void) { return g_err.c_str(); }

}  // extern "C"
