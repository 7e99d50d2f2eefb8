// Internal declarations of the gfx950 sparse-voxel rasterizer library.
// Device structures, the workspace layout and the kernel launchers shared by
// the translation units.  Not part of the public ABI (include/svraster.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "svraster.h"

namespace svr {

constexpr int kBlock = 256;       // threads per workgroup: 4 wave64
constexpr uint32_t kBigEmit = 64;    // entries above which a voxel is emitted by whole workgroups
constexpr uint32_t kBigChunk = 512;  // tiles of such a voxel per item of the whole-grid pass
constexpr int kScanItems = 16;
constexpr int kScanTile = kBlock * kScanItems;  // counts per scan block
constexpr int kSortItems = 16;
constexpr int kSortPart = kBlock * kSortItems;  // (key, value) pairs per sort partition
// frames of at most kCountTiles tiles whose keys are unique within a tile are
// bucketed by tile with a counting sort (a per-tile histogram in LDS)
constexpr int kCountTiles = 32768;
constexpr float kZNear = 1e-4f;   // corners closer than this to the camera plane
                                  // make a voxel cover every tile
constexpr int kVidBits = 29;
constexpr uint32_t kVidMask = (1u << kVidBits) - 1u;

// A camera as the kernels see it.  Rotation is world-to-camera (row-major);
// `o` is the camera centre in world space.
struct DevCam {
  double od[3];       // camera centre in fp64 (ray origin of the render passes)
  float r[9];
  float o[3];
  float fx, fy, cx, cy;
  int32_t W, H, ntx, nty;
  int32_t tile_off;   // first global tile id of this camera
  int32_t sat_off;    // offset of this camera's (nty+1) x (ntx+1) summed-area table
  int64_t pix_off;    // first pixel of this camera in the per-pixel arrays
};

struct CamSet {
  int32_t n;
  int32_t total_tiles;
  int32_t tile;       // tile edge in pixels (8, 16 or 32)
  int32_t tshift;     // log2(tile)
  DevCam c[SVR_MAX_CAMERAS];
};

// Per view-voxel record written by the projection pass and read by the
// render passes, 64 bytes:
//   q0 = voxel centre xyz, edge length
//   q1 = raw densities of corners 0..3, q2 = corners 4..7
//   q3 = clamped SH colour rgb, bits of the channels with a positive
//        pre-clamp value (as int)
struct alignas(16) VoxRec {
  float4 q0, q1, q2, q3;
};

// Workspace header (device): counters written by kernels.
// tiles are rendered heaviest first, in buckets of floor(log2(entries))
constexpr int kOrderBuckets = 16;
// the backward of a tile with more entries than this runs as several chunks
// of this many entries, one workgroup each (a multiple of every batch size)
constexpr int kBwdChunk = 256;
constexpr uint32_t kNoSplit = 0xffffffffu;
// workgroups that take the split chunks (each loops over several)
constexpr int kSplitWgs = 2048;

struct WsHeader {
  unsigned long long n_entries;   // E (may exceed capacity)
  uint32_t overflow;              // E > capacity seen by the emitter
  uint32_t error;                 // bit 0: sort look-back spin limit hit; bit 1: chunk list full;
                                  // bit 2: tile counts disagree with the entry count
  uint32_t tickets[16];           // sort partition tickets, one per pass
  unsigned long long stats[8];    // render statistics (svr_render_stats)
  uint32_t work[8];               // persistent render: work[0] counts taken positions
  uint32_t big_count;             // voxels queued for the whole-grid emission pass
  uint32_t pad[19];
};
static_assert(sizeof(WsHeader) == 256, "header size");

struct Layout {
  // sizes
  int64_t N, NV, cap, P;
  int32_t n_cams, T, sat_total, key_bits, passes, L;
  int32_t key_low;  // bits below the tile id: 3L + 3 (path key) or log2 of the rank range
  int32_t count_sort;  // 1: entries bucketed by tile with the counting sort, else radix passes
  int32_t tile, tshift, persistent;
  int64_t scan_blocks, sort_parts;
  // byte offsets into the workspace
  size_t hdr, count, rect, rec, scan_part;
  size_t tile_mask, tile_sat, tile_range, tile_order, tile_rank;
  size_t tile_count;  // per tile: entry count, then the next free position (counting sort)
  size_t split_base, split_items, ckpt;  // backward chunks of heavy tiles
  size_t big_list;                       // (view-voxel, first output) of voxels emitted by
  int64_t max_big;                       // the whole-grid pass; its capacity
  size_t ckpt_aux;                       // the same for depth and normal
  size_t g_nrm;                          // per voxel dL/dn (normal images)
  int64_t max_split;                     // capacity of the chunk list (>= sum of splits)
  size_t keys0, keys1, vals0, vals1;
  size_t sort_hist, sort_status0, sort_status1;
  size_t px_tau, px_last;
  size_t g_corner, g_rgb;
  size_t total;
};

// ---- device helpers shared by the mask and render kernels ----------------
// World direction (not normalised) of the ray through the centre of pixel
// (u, v).  Written with explicit fused multiply-adds so every kernel that
// calls it computes bit-identical directions (and hence sign patterns).
__device__ __forceinline__ void pixel_dir(const DevCam& c, int u, int v, float& dx, float& dy,
                                          float& dz) {
  float x = ((float)u + 0.5f - c.cx) / c.fx;
  float y = ((float)v + 0.5f - c.cy) / c.fy;
  dx = __fmaf_rn(c.r[0], x, __fmaf_rn(c.r[3], y, c.r[6]));
  dy = __fmaf_rn(c.r[1], x, __fmaf_rn(c.r[4], y, c.r[7]));
  dz = __fmaf_rn(c.r[2], x, __fmaf_rn(c.r[5], y, c.r[8]));
}

// The same ray in fp64, normalised: the geometry of the render passes (ray-box
// test and sample positions) runs in double precision, so the segment length
// of a grazing hit keeps its relative precision.
__device__ __forceinline__ void pixel_dir_f64(const DevCam& c, int u, int v, double& dx, double& dy,
                                              double& dz) {
  const double x = ((double)u + 0.5 - (double)c.cx) / (double)c.fx;
  const double y = ((double)v + 0.5 - (double)c.cy) / (double)c.fy;
  dx = (double)c.r[0] * x + (double)c.r[3] * y + (double)c.r[6];
  dy = (double)c.r[1] * x + (double)c.r[4] * y + (double)c.r[7];
  dz = (double)c.r[2] * x + (double)c.r[5] * y + (double)c.r[8];
  const double n = 1.0 / sqrt(dx * dx + dy * dy + dz * dz);
  dx *= n; dy *= n; dz *= n;
}

__device__ __forceinline__ int sign_bits(float dx, float dy, float dz) {
  return (dx < 0.f ? 4 : 0) | (dy < 0.f ? 2 : 0) | (dz < 0.f ? 1 : 0);
}

// ---- launchers (all asynchronous on `s`) ----------------------------------
// preprocess
// Logical block of workgroup b when the grid has 8 * ceil(nblocks / 8)
// workgroups: workgroups are dealt to the 8 XCDs round-robin, so this gives
// each XCD a contiguous range of logical blocks (neighbouring blocks then share
// that XCD's L2).  Returns >= nblocks for the padding workgroups.
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t nblocks) {
  const int64_t per = (nblocks + 7) >> 3;
  return (b & 7) * per + (b >> 3);
}

// order LDS accesses between the lanes of one wave (no workgroup barrier)
__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s);

// several arrays zeroed by one kernel launch (at most kFillRegions, in order)
constexpr int kFillRegions = 4;
struct FillSet {
  uint32_t* p[kFillRegions] = {nullptr, nullptr, nullptr, nullptr};
  int64_t n[kFillRegions] = {0, 0, 0, 0};
  int64_t total = 0;
  int k = 0;
  void add(uint32_t* ptr, int64_t count);
};
hipError_t launch_zero_u32(const FillSet& f, hipStream_t s);
hipError_t launch_tile_masks(const CamSet& cams, uint8_t* mask, uint2* range, uint32_t* count,
                             hipStream_t s);
hipError_t launch_tile_sat(const CamSet& cams, const uint8_t* mask, uint32_t* sat, hipStream_t s);
hipError_t launch_project(const svr_scene& sc, const CamSet& cams, const Layout& L, void* ws,
                          hipStream_t s);
hipError_t launch_scan(const Layout& L, void* ws, hipStream_t s);
hipError_t launch_emit(const svr_scene& sc, const CamSet& cams, const Layout& L, void* ws,
                       hipStream_t s);
// sort
size_t sort_scratch_bytes(int64_t n, int bits, int64_t* parts_out);
hipError_t launch_radix_sort(uint64_t* k0, uint32_t* v0, uint64_t* k1, uint32_t* v1,
                             const unsigned long long* n_dev, int64_t n_max, int key_bits, int lo,
                             uint32_t* hist, uint32_t* st0, uint32_t* st1, uint32_t* tickets,
                             uint32_t* err, bool* result_in_1, hipStream_t s);
hipError_t launch_tile_sort(const Layout& L, void* ws, uint64_t* keys, uint32_t* vals, uint64_t* ktmp,
                            uint32_t* vtmp, hipStream_t s);
hipError_t launch_tile_ranges(const Layout& L, void* ws, const uint64_t* keys, hipStream_t s);
hipError_t launch_tile_count_sort(const Layout& L, void* ws, int64_t n_max, hipStream_t s);
size_t order_rank_scratch_bytes(int64_t N, int L);
hipError_t launch_order_ranks(const uint64_t* octpath, int64_t N, int L, uint32_t* rank,
                              void* scratch, hipStream_t s);
hipError_t launch_grid_adjacency(const int32_t* vox_grid, int64_t N, int64_t M, int32_t* adj_off,
                                 int32_t* adj, void* scratch, hipStream_t s);
size_t grid_adjacency_scratch_bytes(int64_t N, int64_t M);
// render
hipError_t launch_render_fwd(const svr_scene& sc, const CamSet& cams, const svr_opts& o,
                             const Layout& L, void* ws, const uint32_t* vals, float* rgba,
                             const svr_extra* extra, hipStream_t s);
hipError_t launch_render_bwd(const svr_scene& sc, const CamSet& cams, const svr_opts& o,
                             const Layout& L, void* ws, const uint32_t* vals,
                             const float* grad_rgba, const svr_extra* extra, hipStream_t s);
hipError_t launch_sh_bwd(const svr_scene& sc, const CamSet& cams, const Layout& L, void* ws,
                         float* grad_grid, float* grad_sh, bool accumulate, bool aux,
                         hipStream_t s);

// ---- diagnostics: kernel timing ------------------------------------------
// When enabled (svr_timing_enable), every launch is bracketed by HIP events
// recorded on the launch stream; svr_timing_read aggregates them per kernel.
int timing_begin(hipStream_t s);
void timing_end(int slot, const char* name, hipStream_t s);

#define SVR_LAUNCH(name, kern, grid, block, shmem, stream, ...)            \
  do {                                                                     \
    const int slot_ = ::svr::timing_begin(stream);                         \
    hipLaunchKernelGGL(kern, grid, block, shmem, stream, __VA_ARGS__);     \
    ::svr::timing_end(slot_, name, stream);                                \
  } while (0)

hipError_t launch_count_inview(const Layout& L, void* ws, hipStream_t s);
hipError_t launch_atomic_probe(float* corner, float* colour, int64_t n_rows, int64_t n_waves,
                               int iters, hipStream_t s);
hipError_t launch_downsample(const float* in, int w_in, int h_in, float* out, int w_out,
                             int h_out, const float bg[3], hipStream_t s);
hipError_t launch_downsample_bwd(const float* gout, int w_out, int h_out, float* gin, int w_in,
                                 int h_in, const float bg[3], hipStream_t s);

// svr_mesh.hip
// Camera of the TSDF fusion: projection by the world-to-camera matrix as
// given (R p + t), distances from the fp64 centre -R^T t.
struct FuseCam {
  double od[3];
  float r[9];
  float t[3];
  float fx, fy, cx, cy;
  int32_t W, H;
  int64_t pix_off;
};
struct FuseCamSet {
  int32_t n;
  FuseCam c[SVR_MAX_CAMERAS];
};
hipError_t launch_tsdf_fuse(const float* grid_pos, int64_t M, const FuseCamSet& cams, const float* depth,
                            const float* rgba, float min_alpha, float trunc, float* tsdf,
                            float* weight, const uint32_t* order, bool first, bool last,
                            hipStream_t s);
hipError_t launch_mesh_cells(const svr_scene& sc, const float* field, const float* weight, float iso,
                             int64_t max_tris, int32_t* keys, float* pos, unsigned long long* count,
                             const uint32_t* order, hipStream_t s);
hipError_t launch_morton_keys(const float* pos, int64_t n, const float* lo, float extent,
                              uint64_t* keys, uint32_t* vals, hipStream_t s);
void mesh_case_table(uint8_t* counts, uint8_t* verts);  // [256], [256][36]
hipError_t launch_render_stats(const svr_scene& sc, const CamSet& cams, const svr_opts& o,
                               const Layout& L, void* ws, const uint32_t* vals, hipStream_t s);

template <typename T>
inline T* at(void* ws, size_t off) {
  return reinterpret_cast<T*>(reinterpret_cast<char*>(ws) + off);
}

}  // namespace svr
