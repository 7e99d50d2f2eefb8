// Projection, per-view pre-processing and duplication of voxels per tile
// (Sec. 3.1.2 "Projection to image space" and "Pre-processing voxels";
// Supp. B.1 duplication per tile and ray-sign pattern; Supp. B.2 key).
//
// Passes, all over device-resident data:
//   k_tile_masks   one workgroup per 16x16 tile: OR of the ray-sign patterns
//                  of its in-image pixels (8-bit mask)
//   k_tile_sat     one workgroup per camera: summed-area table of the mask
//                  popcounts, so a voxel counts its entries in O(1)
//   k_project      one thread per (voxel, camera): corner projection, culling,
//                  pixel rectangle, entry count; for counted voxels also the
//                  64-byte render record (box, 8 corner densities, SH colour)
//   k_scan_top     exclusive scan of the per-workgroup entry totals
//   k_emit         the (key, value) entries for every tile of a voxel's
//                  rectangle and every sign pattern present in that tile
#include "svr_internal.h"
#include "svr_sh.h"

namespace svr {

// ---------------------------------------------------------------------------
__global__ void k_fill_u32(uint32_t* __restrict__ p, uint32_t v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + kBlock - 1) / kBlock;
  if (blocks > 8192) blocks = 8192;
  SVR_LAUNCH("fill", k_fill_u32, dim3((unsigned)blocks), dim3(kBlock), 0, s, p, v, n);
  return hipGetLastError();
}

// zero up to kFillRegions arrays in one launch: each workgroup takes a share
// of every array; 16-byte stores over the 16-byte aligned middle of an array
__global__ void k_zero_u32(FillSet f) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int r = 0; r < f.k; ++r) {
    uint32_t* p = f.p[r];
    const int64_t n = f.n[r];
    // head up to the first 16-byte boundary, then uint4 stores, then the tail
    const int64_t head = min(n, (int64_t)(((16u - ((uintptr_t)p & 15u)) & 15u) >> 2));
    const int64_t n4 = (n - head) >> 2;
    if (tid < head) p[tid] = 0u;
    uint4* q = reinterpret_cast<uint4*>(p + head);
    for (int64_t i = tid; i < n4; i += stride) q[i] = make_uint4(0u, 0u, 0u, 0u);
    const int64_t t0 = head + 4 * n4;
    if (tid < n - t0) p[t0 + tid] = 0u;
  }
}

hipError_t launch_zero_u32(const FillSet& f, hipStream_t s) {
  if (f.total <= 0) return hipSuccess;
  int64_t blocks = (f.total + kBlock - 1) / kBlock;
  if (blocks > 8192) blocks = 8192;
  SVR_LAUNCH("fill", k_zero_u32, dim3((unsigned)blocks), dim3(kBlock), 0, s, f);
  return hipGetLastError();
}

void FillSet::add(uint32_t* ptr, int64_t count) {
  if (count <= 0) return;
  p[k] = ptr;
  n[k] = count;
  ++k;
  total += count;
}

__device__ __forceinline__ int find_cam(const CamSet& cams, int gtile) {
  int c = 0;
  for (int i = 1; i < cams.n; ++i)
    if (gtile >= cams.c[i].tile_off) c = i;
  return c;
}

// ---------------------------------------------------------------------------
// Per tile, the OR of 1 << sign_bits over its in-image pixel centres.  A
// workgroup covers kBlock pixels: 4 tiles of 8x8, one of 16x16, or one of
// 32x32 with 4 pixels per thread.
__global__ __launch_bounds__(kBlock) void k_tile_masks(CamSet cams, uint8_t* __restrict__ mask,
                                                       uint2* __restrict__ range,
                                                       uint32_t* __restrict__ count) {
  __shared__ uint32_t m[4];
  const int ts = cams.tile;
  const int tiles_per_wg = ts == 8 ? 4 : 1;
  const int sub = ts == 8 ? (int)threadIdx.x >> 6 : 0;  // tile of this thread in the workgroup
  const int g = (int)blockIdx.x * tiles_per_wg + sub;
  if (threadIdx.x < 4) m[threadIdx.x] = 0;
  __syncthreads();
  if (g < cams.total_tiles) {
    const int ci = find_cam(cams, g);
    const DevCam& c = cams.c[ci];
    const int t = g - c.tile_off;
    const int tx = t % c.ntx, ty = t / c.ntx;
    const int k0 = ts == 8 ? (int)threadIdx.x & 63 : (int)threadIdx.x;
    const int step = ts == 8 ? 64 : kBlock;
    uint32_t mine = 0;
    for (int k = k0; k < ts * ts; k += step) {
      const int u = tx * ts + (k & (ts - 1));
      const int v = ty * ts + (k >> cams.tshift);
      if (u < c.W && v < c.H) {
        float dx, dy, dz;
        pixel_dir(c, u, v, dx, dy, dz);
        mine |= 1u << sign_bits(dx, dy, dz);
      }
    }
    if (mine) atomicOr(&m[sub], mine);
  }
  __syncthreads();
  if (threadIdx.x < (unsigned)tiles_per_wg) {
    const int gt = (int)blockIdx.x * tiles_per_wg + (int)threadIdx.x;
    if (gt < cams.total_tiles) {
      mask[gt] = (uint8_t)m[threadIdx.x];
      range[gt] = make_uint2(0u, 0u);  // tiles without entries keep an empty range
      if (count) count[gt] = 0u;       // entry count of the counting sort
    }
  }
}

hipError_t launch_tile_masks(const CamSet& cams, uint8_t* mask, uint2* range, uint32_t* count,
                             hipStream_t s) {
  const int per = cams.tile == 8 ? 4 : 1;
  SVR_LAUNCH("tile_masks", k_tile_masks, dim3((cams.total_tiles + per - 1) / per), dim3(kBlock), 0,
             s, cams, mask, range, count);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Summed-area table of popcount(mask) per camera:
//   sat[ty * (ntx+1) + tx] = sum over tiles (x < tx, y < ty)
// in two passes: a wave per table row scans popcounts along the row, then a
// wave per 64 columns accumulates down the rows.

// camera and local index of global item `i` of a per-camera sequence whose
// camera c holds n(c) items
template <typename F>
__device__ __forceinline__ int split_by_cam(const CamSet& cams, int64_t i, F n, int64_t& local) {
  int64_t base = 0;
  for (int c = 0; c < cams.n; ++c) {
    const int64_t nc = n(cams.c[c]);
    if (i < base + nc) {
      local = i - base;
      return c;
    }
    base += nc;
  }
  return -1;
}

__global__ __launch_bounds__(kBlock) void k_sat_rows(CamSet cams, const uint8_t* __restrict__ mask,
                                                     uint32_t* __restrict__ sat) {
  const int64_t wv = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
  const int lane = (int)threadIdx.x & 63;
  int64_t ty;
  const int ci = split_by_cam(cams, wv, [](const DevCam& c) { return (int64_t)c.nty + 1; }, ty);
  if (ci < 0) return;
  const DevCam& c = cams.c[ci];
  const int W1 = c.ntx + 1;
  uint32_t* S = sat + c.sat_off + ty * W1;
  if (lane == 0) S[0] = 0;
  const uint8_t* Mk = mask + c.tile_off + (ty - 1) * c.ntx;
  uint32_t carry = 0;
  for (int x0 = 0; x0 < c.ntx; x0 += 64) {
    const int tx = x0 + lane;
    uint32_t v = (ty > 0 && tx < c.ntx) ? (uint32_t)__popc((unsigned)Mk[tx]) : 0u;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t t = __shfl_up(v, o, 64);
      if (lane >= o) v += t;
    }
    if (tx < c.ntx) S[tx + 1] = carry + v;
    carry += __shfl(v, 63, 64);
  }
}

__global__ __launch_bounds__(kBlock) void k_sat_cols(CamSet cams, uint32_t* __restrict__ sat) {
  const int64_t wv = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
  const int lane = (int)threadIdx.x & 63;
  int64_t blk;
  const int ci = split_by_cam(cams, wv, [](const DevCam& c) { return (int64_t)(c.ntx + 1 + 63) / 64; },
                              blk);
  if (ci < 0) return;
  const DevCam& c = cams.c[ci];
  const int W1 = c.ntx + 1;
  const int tx = (int)blk * 64 + lane;
  if (tx >= W1) return;
  uint32_t* S = sat + c.sat_off + tx;
  // 16 rows per step: the loads are issued together, then summed and stored
  constexpr int kRows = 16;
  uint32_t acc = 0;
  for (int y0 = 0; y0 <= c.nty; y0 += kRows) {
    uint32_t v[kRows];
#pragma unroll
    for (int k = 0; k < kRows; ++k) v[k] = y0 + k <= c.nty ? S[(int64_t)(y0 + k) * W1] : 0u;
#pragma unroll
    for (int k = 0; k < kRows; ++k) {
      acc += v[k];
      if (y0 + k <= c.nty) S[(int64_t)(y0 + k) * W1] = acc;
    }
  }
}

hipError_t launch_tile_sat(const CamSet& cams, const uint8_t* mask, uint32_t* sat, hipStream_t s) {
  int64_t rows = 0, colblocks = 0;
  for (int i = 0; i < cams.n; ++i) {
    rows += cams.c[i].nty + 1;
    colblocks += (cams.c[i].ntx + 1 + 63) / 64;
  }
  const int wpb = kBlock / 64;
  SVR_LAUNCH("tile_sat", k_sat_rows, dim3((unsigned)((rows + wpb - 1) / wpb)), dim3(kBlock), 0, s,
             cams, mask, sat);
  SVR_LAUNCH("tile_sat", k_sat_cols, dim3((unsigned)((colblocks + wpb - 1) / wpb)), dim3(kBlock), 0,
             s, cams, sat);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
template <int D>
__device__ __forceinline__ void sh_color(const float* __restrict__ shv, float dx, float dy, float dz,
                                         float rgb[3], uint32_t& pos_bits) {
  constexpr int NB = (D + 1) * (D + 1);
  float Y[16];
  sh_basis<D>(dx, dy, dz, Y);
  float acc[3] = {0.f, 0.f, 0.f};
  if (D == 3) {
    const float4* s4 = reinterpret_cast<const float4*>(shv);
    float buf[48];
#pragma unroll
    for (int i = 0; i < 12; ++i) {
      const float4 q = s4[i];
      buf[4 * i + 0] = q.x; buf[4 * i + 1] = q.y; buf[4 * i + 2] = q.z; buf[4 * i + 3] = q.w;
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      acc[0] = __fmaf_rn(buf[3 * j + 0], Y[j], acc[0]);
      acc[1] = __fmaf_rn(buf[3 * j + 1], Y[j], acc[1]);
      acc[2] = __fmaf_rn(buf[3 * j + 2], Y[j], acc[2]);
    }
  } else {
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      acc[0] = __fmaf_rn(shv[3 * j + 0], Y[j], acc[0]);
      acc[1] = __fmaf_rn(shv[3 * j + 1], Y[j], acc[1]);
      acc[2] = __fmaf_rn(shv[3 * j + 2], Y[j], acc[2]);
    }
  }
  pos_bits = 0;
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) {
    if (acc[ch] > 0.f) pos_bits |= 1u << ch;
    rgb[ch] = fmaxf(acc[ch], 0.f);
  }
}

// SH colour (degree 3) from the voxel's 48 coefficients staged in LDS as 12
// float4 (Sec. 3.1.1 eq. vox_color, clamped at 0)
__device__ __forceinline__ void sh_color3_lds(const float4* __restrict__ s4, float dx, float dy,
                                              float dz, float rgb[3], uint32_t& pos_bits) {
  float Y[16];
  sh_basis<3>(dx, dy, dz, Y);
  // each 16-byte piece is used as it arrives (coefficient f = 3 j + channel),
  // so few registers are held; the sums run in the same order as above
  float acc[3] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int i = 0; i < 12; ++i) {
    const float4 q = s4[i];
    const float v[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int f = 4 * i + c;
      acc[f % 3] = __fmaf_rn(v[c], Y[f / 3], acc[f % 3]);
    }
  }
  pos_bits = 0;
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) {
    if (acc[ch] > 0.f) pos_bits |= 1u << ch;
    rgb[ch] = fmaxf(acc[ch], 0.f);
  }
}

// degree-3 SH staging: a wave copies the coefficients of kShStageVox
// consecutive voxels (contiguous in memory) into LDS with coalesced float4
// loads, rows padded to 13 float4 so that the lanes' 16-byte reads of
// different voxels fall in different banks
constexpr int kShStageVox = 32;
constexpr int kShRow = 13;

__device__ __forceinline__ uint32_t sat_rect(const uint32_t* __restrict__ S, int W1, int tx0,
                                             int tx1, int ty0, int ty1) {
  return S[(ty1 + 1) * W1 + tx1 + 1] - S[ty0 * W1 + tx1 + 1] - S[(ty1 + 1) * W1 + tx0] +
         S[ty0 * W1 + tx0];
}

__device__ __forceinline__ unsigned long long wave_incl_scan(unsigned long long v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    unsigned long long t = __shfl_up(v, d, 64);
    if (lane >= d) v += t;
  }
  return v;
}

__device__ __forceinline__ unsigned long long block_excl_scan(unsigned long long v,
                                                              unsigned long long& excl) {
  __shared__ unsigned long long wsum[kBlock / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  unsigned long long inc = wave_incl_scan(v);
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  unsigned long long base = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < kBlock / 64; ++i) {
    if (i < w) base += wsum[i];
    tot += wsum[i];
  }
  excl = base + inc - v;
  __syncthreads();
  return tot;
}

// ---------------------------------------------------------------------------
// key = global tile << (3L + 3) | (top 3L path bits XOR s repeated) << 3 | s
//       (the direction-dependent Morton order of Supp. B.2 as one XOR)
// value = s << 29 | voxel id
// A voxel's entries are its rectangle's tiles in row-major order, each tile
// with the sign patterns present in it in ascending order.

struct EmitCtx {
  uint64_t top, rep;
  int sh;
  uint32_t vid;
  bool ranked;    // key low bits from the order ranks (else from the path)
  uint4 r03, r47;  // the voxel's 8 order ranks, loaded together up front
};

__device__ __forceinline__ EmitCtx emit_ctx(const uint64_t* __restrict__ octpath,
                                            const uint32_t* __restrict__ rank, int64_t vid, int L,
                                            uint64_t rep, int sh) {
  EmitCtx e;
  e.top = octpath[vid] >> (3 * (SVR_MAX_LEVELS - L));
  e.rep = rep;
  e.sh = sh;
  e.vid = (uint32_t)vid;
  e.ranked = rank != nullptr;
  if (e.ranked) {
    const uint4* r = reinterpret_cast<const uint4*>(rank + vid * 8);
    e.r03 = r[0];
    e.r47 = r[1];
  } else {
    e.r03 = e.r47 = make_uint4(0u, 0u, 0u, 0u);
  }
  return e;
}

__device__ __forceinline__ uint32_t rank_of(const EmitCtx& e, int sgn) {
  const uint4 q = sgn < 4 ? e.r03 : e.r47;
  const int i = sgn & 3;
  return i < 2 ? (i == 0 ? q.x : q.y) : (i == 2 ? q.z : q.w);
}

__device__ __forceinline__ void emit_tile(const EmitCtx& e, int gt, uint32_t m,
                                          unsigned long long o, int64_t cap,
                                          uint64_t* __restrict__ keys, uint32_t* __restrict__ vals) {
  while (m) {
    const int sgn = __ffs(m) - 1;
    m &= m - 1;
    if (o < (unsigned long long)cap) {
      const uint64_t low = e.ranked ? (uint64_t)rank_of(e, sgn)
                                    : ((e.top ^ ((uint64_t)sgn * e.rep)) << 3) | (uint64_t)sgn;
      keys[o] = ((uint64_t)gt << e.sh) | low;
      vals[o] = ((uint32_t)sgn << kVidBits) | e.vid;
    }
    ++o;
  }
}

// ONE: a single camera, whose parameters are then wave-uniform (scalar
// loads) instead of per-lane reads of the camera array
template <int D, bool ONE>
__global__ __launch_bounds__(kBlock) void k_project(
    int64_t NV, int n_cams, CamSet cams, const float* __restrict__ center,
    const float* __restrict__ size, const int32_t* __restrict__ vox_grid,
    const float* __restrict__ grid_raw, const float* __restrict__ sh, int64_t N,
    const uint32_t* __restrict__ sat, uint32_t* __restrict__ count, uint2* __restrict__ rect,
    VoxRec* __restrict__ rec, unsigned long long* __restrict__ part) {
  __shared__ float4 shs[D == 3 ? kBlock / 64 : 1][D == 3 ? kShStageVox * kShRow : 1];
  const int64_t vv0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool active = vv0 < NV;
  const int64_t vv = active ? vv0 : NV - 1;  // inactive lanes stay for the wave-wide staging
  const int64_t vid = ONE ? vv : vv / n_cams;
  const int ci = ONE ? 0 : (int)(vv - vid * n_cams);
  const DevCam& c = cams.c[ci];
  // the corner densities are gathered first (also for voxels that turn out
  // culled), so their reads overlap the projection instead of ending it
  const int4* vg = reinterpret_cast<const int4*>(vox_grid + vid * 8);
  const int4 ga = vg[0], gb = vg[1];
  const float4 q1 = make_float4(grid_raw[ga.x], grid_raw[ga.y], grid_raw[ga.z], grid_raw[ga.w]);
  const float4 q2 = make_float4(grid_raw[gb.x], grid_raw[gb.y], grid_raw[gb.z], grid_raw[gb.w]);
  const float s = size[vid];
  const float h = 0.5f * s;
  // centre relative to the camera, then camera-space centre Pc = R (centre - o)
  const float rx = center[vid] - c.o[0];
  const float ry = center[N + vid] - c.o[1];
  const float rz = center[2 * N + vid] - c.o[2];
  float P[3], A[3][3];  // A[r][j] = h * R[r][j]: half-edge vectors in camera space
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    P[r] = c.r[3 * r + 0] * rx + c.r[3 * r + 1] * ry + c.r[3 * r + 2] * rz;
#pragma unroll
    for (int j = 0; j < 3; ++j) A[r][j] = h * c.r[3 * r + j];
  }
  // support of the box along a camera-space direction n: n.P + sum_j |n.A_j|
  auto support = [&](float nx, float ny, float nz) {
    float m = nx * P[0] + ny * P[1] + nz * P[2];
#pragma unroll
    for (int j = 0; j < 3; ++j) m += fabsf(nx * A[0][j] + ny * A[1][j] + nz * A[2][j]);
    return m;
  };
  const float W = (float)c.W, H = (float)c.H;
  bool culled = support(0.f, 0.f, 1.f) <= 0.f ||                 // every corner behind
                support(c.fx, 0.f, c.cx) < 0.f ||                 // left of the image
                support(-c.fx, 0.f, W - c.cx) < 0.f ||            // right
                support(0.f, c.fy, c.cy) < 0.f ||                 // above
                support(0.f, -c.fy, H - c.cy) < 0.f;              // below
  uint32_t cnt = 0;
  int u0 = 0, u1 = -1, v0 = 0, v1 = -1;
  if (!culled) {
    const float zmin = -support(0.f, 0.f, -1.f);
    if (zmin < kZNear) {
      u0 = 0; u1 = c.W - 1; v0 = 0; v1 = c.H - 1;
    } else {
      float x0 = 3.0e38f, x1 = -3.0e38f, y0 = 3.0e38f, y1 = -3.0e38f;
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const float sx = (k & 4) ? 1.f : -1.f, sy = (k & 2) ? 1.f : -1.f, sz = (k & 1) ? 1.f : -1.f;
        const float X = P[0] + sx * A[0][0] + sy * A[0][1] + sz * A[0][2];
        const float Y = P[1] + sx * A[1][0] + sy * A[1][1] + sz * A[1][2];
        const float Z = P[2] + sx * A[2][0] + sy * A[2][1] + sz * A[2][2];
        const float iz = 1.f / Z;
        const float x = c.fx * X * iz + c.cx;
        const float y = c.fy * Y * iz + c.cy;
        x0 = fminf(x0, x); x1 = fmaxf(x1, x); y0 = fminf(y0, y); y1 = fmaxf(y1, y);
      }
      // pixel (u, v) is covered when its centre lies in the box; a small
      // dilation keeps the fp32 box conservative
      const float eps = 1.f / 256.f;
      x0 = fminf(fmaxf(x0, -2.f), W + 2.f); x1 = fminf(fmaxf(x1, -2.f), W + 2.f);
      y0 = fminf(fmaxf(y0, -2.f), H + 2.f); y1 = fminf(fmaxf(y1, -2.f), H + 2.f);
      u0 = max((int)ceilf(x0 - 0.5f - eps), 0);
      u1 = min((int)floorf(x1 - 0.5f + eps), c.W - 1);
      v0 = max((int)ceilf(y0 - 0.5f - eps), 0);
      v1 = min((int)floorf(y1 - 0.5f + eps), c.H - 1);
    }
    if (u0 <= u1 && v0 <= v1) {
      cnt = sat_rect(sat + c.sat_off, c.ntx + 1, u0 >> cams.tshift, u1 >> cams.tshift,
                     v0 >> cams.tshift, v1 >> cams.tshift);
    }
  }
  if (!active) cnt = 0;
  {
    // the workgroup's entry total, for the scan of the offsets
    unsigned long long ex;
    const unsigned long long tot = block_excl_scan(cnt, ex);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
  }
  if (active) {
    count[vv] = cnt;
    rect[vv] = cnt == 0 ? make_uint2(1u, 0u)
                        : make_uint2((uint32_t)u0 | ((uint32_t)u1 << 16),
                                     (uint32_t)v0 | ((uint32_t)v1 << 16));
  }
  const bool need = cnt > 0;
  // pre-process: SH colour for the direction camera centre -> voxel centre,
  // then gather the 8 corner densities
  const float rn = rsqrtf(rx * rx + ry * ry + rz * rz);
  float rgb[3] = {0.f, 0.f, 0.f};
  uint32_t bits = 0;
  if (D == 3) {
    const unsigned long long needm = __ballot(need);
    if (needm == 0ull) return;
    const int lane = (int)threadIdx.x & 63, w = (int)threadIdx.x >> 6;
    // the wave's voxels: [vlo, vhi] (ids grow with the lane)
    const int64_t vlo = __shfl(vid, 0, 64);
    const int64_t vhi = __shfl(vid, 63, 64);
    const float4* sh4 = reinterpret_cast<const float4*>(sh);
    float4* S = shs[w];
    // one round stages kShStageVox voxels, kPer float4 per lane; the next
    // round's reads are issued before the current round is evaluated
    constexpr int kPer = kShStageVox * 12 / 64;
    float4 buf[kPer];
    auto round_reads = [&](int64_t vb) {
      const int nv = (int)min((int64_t)kShStageVox, vhi - vb + 1);
      // with one camera, lane L holds voxel vlo + L: rows of voxels that
      // emit nothing are not read
      const unsigned long long rows = n_cams == 1 ? (needm >> (vb - vlo)) : ~0ull;
#pragma unroll
      for (int i = 0; i < kPer; ++i) {
        const int q = lane + 64 * i;
        buf[i] = (q < nv * 12 && ((rows >> (q / 12)) & 1ull)) ? sh4[vb * 12 + q]
                                                              : make_float4(0.f, 0.f, 0.f, 0.f);
      }
    };
    round_reads(vlo);
    for (int64_t vb = vlo; vb <= vhi; vb += kShStageVox) {
      const int nv = (int)min((int64_t)kShStageVox, vhi - vb + 1);
#pragma unroll
      for (int i = 0; i < kPer; ++i) {
        const int q = lane + 64 * i;
        if (q < nv * 12) S[(q / 12) * kShRow + q % 12] = buf[i];
      }
      wave_sync_lds();
      if (vb + kShStageVox <= vhi) round_reads(vb + kShStageVox);
      if (need && vid >= vb && vid < vb + nv)
        sh_color3_lds(S + (vid - vb) * kShRow, rx * rn, ry * rn, rz * rn, rgb, bits);
      wave_sync_lds();
    }
  } else if (need) {
    sh_color<D>(sh + vid * (int64_t)(3 * (D + 1) * (D + 1)), rx * rn, ry * rn, rz * rn, rgb,
                bits);
  }
  if (!need) return;
  VoxRec R;
  R.q0 = make_float4(center[vid], center[N + vid], center[2 * N + vid], s);
  R.q1 = q1;
  R.q2 = q2;
  R.q3 = make_float4(rgb[0], rgb[1], rgb[2], __uint_as_float(bits));
  rec[vv] = R;
}

// statistics: number of in-view (voxel, camera) pairs (count > 0), summed per
// workgroup, one atomic per workgroup
__global__ __launch_bounds__(kBlock) void k_count_inview(const uint32_t* __restrict__ count,
                                                         int64_t n, unsigned long long* out) {
  __shared__ unsigned long long part[kBlock / 64];
  unsigned long long c = 0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlock)
    c += count[i] > 0u ? 1ull : 0ull;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
    for (int w = 0; w < kBlock / 64; ++w) t += part[w];
    if (t) atomicAdd(out, t);
  }
}

hipError_t launch_count_inview(const Layout& L, void* ws, hipStream_t s) {
  unsigned long long* out = &at<WsHeader>(ws, L.hdr)->stats[3];
  hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t*>(out), 0u, 2, s);
  if (e != hipSuccess || L.NV == 0) return e;
  int64_t blocks = (L.NV + kBlock * 16 - 1) / (kBlock * 16);
  if (blocks > 1024) blocks = 1024;
  SVR_LAUNCH("count_inview", k_count_inview, dim3((unsigned)blocks), dim3(kBlock), 0, s,
             at<uint32_t>(ws, L.count), L.NV, out);
  return hipGetLastError();
}

hipError_t launch_project(const svr_scene& sc, const CamSet& cams, const Layout& L, void* ws,
                          hipStream_t s) {
  if (L.NV == 0) return hipSuccess;
  dim3 grid((unsigned)((L.NV + kBlock - 1) / kBlock));
  auto* sat = at<uint32_t>(ws, L.tile_sat);
  auto* count = at<uint32_t>(ws, L.count);
  auto* rect = at<uint2>(ws, L.rect);
  auto* rec = at<VoxRec>(ws, L.rec);
  auto* part = at<unsigned long long>(ws, L.scan_part);
#define SVR_PROJ(D)                                                                              \
  if (L.n_cams == 1)                                                                             \
    SVR_LAUNCH("project", (k_project<D, true>), grid, dim3(kBlock), 0, s, L.NV, L.n_cams, cams,  \
               sc.center, sc.size, sc.vox_grid, sc.grid_raw, sc.sh, L.N, sat, count, rect, rec, part); \
  else                                                                                           \
    SVR_LAUNCH("project", (k_project<D, false>), grid, dim3(kBlock), 0, s, L.NV, L.n_cams, cams, \
               sc.center, sc.size, sc.vox_grid, sc.grid_raw, sc.sh, L.N, sat, count, rect, rec, part)
  switch (sc.sh_degree) {
    case 0: SVR_PROJ(0); break;
    case 1: SVR_PROJ(1); break;
    case 2: SVR_PROJ(2); break;
    default: SVR_PROJ(3); break;
  }
#undef SVR_PROJ
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// exclusive scan of the per view-voxel counts into 64-bit offsets


// block-wide exclusive scan of one value per thread; returns the block total

// exclusive scan of the per-workgroup entry totals (in place), kScanItems
// consecutive totals per thread and round; the grand total is the entry count
__global__ __launch_bounds__(kBlock) void k_scan_top(unsigned long long* __restrict__ part, int64_t nb,
                                                     WsHeader* __restrict__ hdr) {
  unsigned long long carry = 0;
  for (int64_t b0 = 0; b0 < nb; b0 += kScanTile) {
    const int64_t j0 = b0 + (int64_t)threadIdx.x * kScanItems;
    unsigned long long v[kScanItems];
    unsigned long long acc = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
      v[i] = j0 + i < nb ? part[j0 + i] : 0ull;
      acc += v[i];
    }
    unsigned long long ex;
    const unsigned long long tot = block_excl_scan(acc, ex);
    ex += carry;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
      if (j0 + i < nb) part[j0 + i] = ex;
      ex += v[i];
    }
    carry += tot;
  }
  if (threadIdx.x == 0) {
    hdr->n_entries = carry;
    hdr->overflow = 0;
    hdr->error = 0;  // the frame's sort and tile order report into it
    hdr->big_count = 0u;
  }
}

hipError_t launch_scan(const Layout& L, void* ws, hipStream_t s) {
  auto* part = at<unsigned long long>(ws, L.scan_part);
  auto* hdr = at<WsHeader>(ws, L.hdr);
  SVR_LAUNCH("scan_top", k_scan_top, dim3(1), dim3(kBlock), 0, s, part, L.scan_blocks, hdr);
  return hipGetLastError();
}


// The workgroup's entries are written in three ways.  A voxel whose tiles
// each hold one sign pattern (count = tiles in its rectangle, the common
// case) has entry j at tile j of its rectangle in row-major order: those
// entries are spread over the whole workgroup, 256 consecutive output
// positions per round, each thread finding its voxel by a binary search over
// the workgroup's offsets in LDS (full lanes, coalesced stores).  The other
// voxels (tiles that several sign patterns share) and the voxels of more
// than kBigEmit entries are queued for k_emit_big, where the whole grid takes
// them a wave per item (they cluster in a Z-curve order: near the lines where
// a ray component changes sign, and in the coarse background levels, and one
// workgroup taking them one after another would set the kernel's length).
// ONE: a single camera (wave-uniform camera parameters).
template <bool ONE>
__global__ __launch_bounds__(kBlock) void k_emit(
    int64_t NV, int n_cams, CamSet cams, const uint64_t* __restrict__ octpath,
    const uint32_t* __restrict__ count, const unsigned long long* __restrict__ part,
    const uint2* __restrict__ rect, const uint8_t* __restrict__ mask,
    const uint32_t* __restrict__ sat, int L, int key_low, const uint32_t* __restrict__ rank,
    int64_t cap, uint64_t* __restrict__ keys, uint32_t* __restrict__ vals,
    WsHeader* __restrict__ hdr, ulonglong2* __restrict__ big, int64_t max_big) {
  __shared__ uint32_t s_off[kBlock + 1];  // offsets in the workgroup, s_off[kBlock] = total
  __shared__ uint32_t s_rx[kBlock];       // tile rectangle: tx0 | ty0 << 16 (simple voxels)
  __shared__ uint32_t s_wd[kBlock];       // its width in tiles; 0: not a simple voxel
  const int64_t vv = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t cnt = vv < NV ? count[vv] : 0u;
  const uint2 r = cnt > 0 ? rect[vv] : make_uint2(1u, 0u);
  // first output position: the workgroup's prefix plus the counts before
  // this thread in the workgroup
  unsigned long long ex;
  const unsigned long long wg_tot = block_excl_scan(cnt, ex);
  const unsigned long long wg_base = part[blockIdx.x];
  const unsigned long long off_vv = wg_base + ex;
  const int sh = key_low;
  const uint64_t rep = ((1ull << (3 * L)) - 1ull) / 7ull;  // 001 001 ... 001 (L triplets)
  const int tx0 = (int)(r.x & 0xffffu) >> cams.tshift, tx1 = (int)(r.x >> 16) >> cams.tshift;
  const int ty0 = (int)(r.y & 0xffffu) >> cams.tshift, ty1 = (int)(r.y >> 16) >> cams.tshift;
  const uint32_t ntiles = cnt > 0 ? (uint32_t)((tx1 - tx0 + 1) * (ty1 - ty0 + 1)) : 0u;
  const bool simple = cnt > 0 && cnt == ntiles;
  if (cnt > 0 && off_vv + cnt > (unsigned long long)cap) atomicOr(&hdr->overflow, 1u);
  // voxels queued for the whole-grid pass: more than kBigEmit entries, or
  // tiles shared by several sign patterns; one item per kBigChunk tiles of
  // the rectangle (a voxel on the near plane covers every tile), reserved
  // with one atomic per wave.  The list holds every item of a frame within
  // the capacity; past it (an overflowing frame) the voxel is emitted here,
  // so that every position below the capacity is written
  const uint32_t nit = (cnt > kBigEmit || (cnt > 0 && !simple))
                           ? (ntiles + kBigChunk - 1) / kBigChunk : 0u;
  bool queued = false;
  {
    const int lane = (int)threadIdx.x & 63;
    uint32_t incl = nit;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t t = __shfl_up(incl, d, 64);
      if (lane >= d) incl += t;
    }
    const uint32_t wtot = __shfl(incl, 63, 64);
    uint32_t wbase = 0;
    if (wtot > 0) {
      if (lane == 63) wbase = atomicAdd(&hdr->big_count, wtot);
      wbase = __shfl(wbase, 63, 64);
    }
    const int64_t q = (int64_t)wbase + (incl - nit);
    queued = nit > 0 && q + nit <= max_big;
    if (queued)
      for (uint32_t k = 0; k < nit; ++k)
        big[q + k] = make_ulonglong2((unsigned long long)vv | ((unsigned long long)k << 40),
                                     off_vv);
  }
  s_off[threadIdx.x] = (uint32_t)ex;
  if (threadIdx.x == kBlock - 1) s_off[kBlock] = (uint32_t)wg_tot;
  s_rx[threadIdx.x] = (uint32_t)tx0 | ((uint32_t)ty0 << 16);
  s_wd[threadIdx.x] = simple && !queued ? (uint32_t)(tx1 - tx0 + 1) : 0u;
  if (cnt > 0 && !simple) {
    if (!queued) {
      const int64_t vid = ONE ? vv : vv / n_cams;
      const DevCam& c = cams.c[ONE ? 0 : (int)(vv - vid * n_cams)];
      const EmitCtx e = emit_ctx(octpath, rank, vid, L, rep, sh);
      unsigned long long o = off_vv;
      for (int ty = ty0; ty <= ty1; ++ty) {
        for (int tx = tx0; tx <= tx1; ++tx) {
          const int gt = c.tile_off + ty * c.ntx + tx;
          const uint32_t m = mask[gt];
          emit_tile(e, gt, m, o, cap, keys, vals);
          o += __popc(m);
        }
      }
    }
  }
  __syncthreads();
  // entry-parallel rounds over the workgroup's output range; positions of
  // voxels that are not simple are skipped (their owners wrote them)
  const uint32_t total = s_off[kBlock];
  if (wg_base + total > (unsigned long long)cap && threadIdx.x == 0) atomicOr(&hdr->overflow, 1u);
  const int64_t vv0 = (int64_t)blockIdx.x * blockDim.x;
  for (uint32_t k = threadIdx.x; k < total; k += kBlock) {
    // owner: the last voxel whose offset is <= k
    int lo = 0;
#pragma unroll
    for (int step = kBlock / 2; step > 0; step >>= 1)
      if (s_off[lo + step] <= k) lo += step;
    const uint32_t wd = s_wd[lo];
    if (wd == 0u) continue;
    const uint64_t o = wg_base + k;
    if (o >= (unsigned long long)cap) continue;
    const uint32_t j = k - s_off[lo];
    const uint32_t row = j / wd;
    const uint32_t rx = s_rx[lo];
    const int64_t ov = vv0 + lo;
    const int64_t vid = ONE ? ov : ov / n_cams;
    const DevCam& c = cams.c[ONE ? 0 : (int)(ov - vid * n_cams)];
    const int gt = c.tile_off + ((int)(rx >> 16) + (int)row) * c.ntx + (int)(rx & 0xffffu) +
                   (int)(j - row * wd);
    uint64_t low;
    int sgn;
    if (rank) {
      // the voxel's 8 order ranks are read beside the tile's mask (one round
      // trip instead of two), then the one of the tile's pattern is taken
      const uint4* rp = reinterpret_cast<const uint4*>(rank + vid * 8);
      const uint4 r03 = rp[0], r47 = rp[1];
      const uint32_t mk = mask[gt];
      // all nine values before any is used: the compiler would otherwise
      // read only the needed rank, after the mask
      asm volatile("" ::"v"(r03.x), "v"(r03.y), "v"(r03.z), "v"(r03.w), "v"(r47.x), "v"(r47.y),
                   "v"(r47.z), "v"(r47.w), "v"(mk));
      sgn = __ffs((int)mk) - 1;
      const uint4 q = sgn < 4 ? r03 : r47;
      const int i = sgn & 3;
      low = (uint64_t)(i < 2 ? (i == 0 ? q.x : q.y) : (i == 2 ? q.z : q.w));
    } else {
      sgn = __ffs((int)mask[gt]) - 1;
      const uint64_t top = octpath[vid] >> (3 * (SVR_MAX_LEVELS - L));
      low = ((top ^ ((uint64_t)sgn * rep)) << 3) | (uint64_t)sgn;
    }
    keys[o] = ((uint64_t)gt << sh) | low;
    vals[o] = ((uint32_t)sgn << kVidBits) | (uint32_t)vid;
  }

}

// the queued voxels: one wave per item (kBigChunk tiles of a voxel's
// rectangle) at a time, one tile per lane, each tile's output offset from
// the summed-area table (or its position, when every tile holds one sign
// pattern)
template <bool ONE>
__global__ __launch_bounds__(kBlock) void k_emit_big(
    int n_cams, CamSet cams, const uint64_t* __restrict__ octpath, const uint2* __restrict__ rect,
    const uint8_t* __restrict__ mask, const uint32_t* __restrict__ sat, int L, int key_low,
    const uint32_t* __restrict__ rank, int64_t cap, uint64_t* __restrict__ keys,
    uint32_t* __restrict__ vals, const WsHeader* __restrict__ hdr,
    const ulonglong2* __restrict__ big, int64_t max_big) {
  const int64_t nq = min((int64_t)hdr->big_count, max_big);
  const int sh = key_low;
  const uint64_t rep = ((1ull << (3 * L)) - 1ull) / 7ull;  // 001 001 ... 001 (L triplets)
  const int lane = (int)threadIdx.x & 63;
  const int64_t nw = (int64_t)gridDim.x * (kBlock / 64);
  for (int64_t q = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6; q < nq; q += nw) {
    const ulonglong2 item = big[q];
    const int64_t bv = (int64_t)(item.x & ((1ull << 40) - 1ull));
    const int chunk = (int)(item.x >> 40);
    const int64_t vid = ONE ? bv : bv / n_cams;
    const DevCam& c = cams.c[ONE ? 0 : (int)(bv - vid * n_cams)];
    const EmitCtx e = emit_ctx(octpath, rank, vid, L, rep, sh);
    const uint2 br = rect[bv];
    const int bx0 = (int)(br.x & 0xffffu) >> cams.tshift, bx1 = (int)(br.x >> 16) >> cams.tshift;
    const int by0 = (int)(br.y & 0xffffu) >> cams.tshift, by1 = (int)(br.y >> 16) >> cams.tshift;
    const int wdt = bx1 - bx0 + 1;
    const int nt = wdt * (by1 - by0 + 1);
    const uint32_t* S = sat + c.sat_off;
    const int W1 = c.ntx + 1;
    const unsigned long long o0 = item.y;
    // one pattern per tile: entry j is tile j; else each tile's offset comes
    // from the summed-area table
    const bool simple = sat_rect(S, W1, bx0, bx1, by0, by1) == (uint32_t)nt;
    const int jend = min(nt, (chunk + 1) * (int)kBigChunk);
    for (int jt = chunk * (int)kBigChunk + lane; jt < jend; jt += 64) {
      const int tx = bx0 + jt % wdt, ty = by0 + jt / wdt;
      unsigned long long o = o0;
      if (simple) {
        o += (unsigned long long)jt;
      } else {
        if (ty > by0) o += sat_rect(S, W1, bx0, bx1, by0, ty - 1);
        if (tx > bx0) o += sat_rect(S, W1, bx0, tx - 1, ty, ty);
      }
      const int gt = c.tile_off + ty * c.ntx + tx;
      emit_tile(e, gt, mask[gt], o, cap, keys, vals);
    }
  }
}

hipError_t launch_emit(const svr_scene& sc, const CamSet& cams, const Layout& L, void* ws,
                       hipStream_t s) {
  if (L.NV == 0) return hipSuccess;
  const bool one = L.n_cams == 1;
  SVR_LAUNCH("emit", one ? k_emit<true> : k_emit<false>,
             dim3((unsigned)((L.NV + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, L.NV, L.n_cams, cams,
             sc.octpath, at<uint32_t>(ws, L.count), at<unsigned long long>(ws, L.scan_part),
             at<uint2>(ws, L.rect), at<uint8_t>(ws, L.tile_mask), at<uint32_t>(ws, L.tile_sat), L.L,
             L.key_low, sc.order_rank, L.cap, at<uint64_t>(ws, L.keys0), at<uint32_t>(ws, L.vals0),
             at<WsHeader>(ws, L.hdr), at<ulonglong2>(ws, L.big_list), L.max_big);
  // the queued voxels, over a grid of fixed size (the count stays on the
  // device, so the launch can be captured in a graph)
  const int64_t gb = L.max_big < 1024 ? L.max_big : 1024;
  SVR_LAUNCH("emit_big", one ? k_emit_big<true> : k_emit_big<false>, dim3((unsigned)gb), dim3(kBlock),
             0, s, L.n_cams, cams, sc.octpath, at<uint2>(ws, L.rect), at<uint8_t>(ws, L.tile_mask),
             at<uint32_t>(ws, L.tile_sat), L.L, L.key_low, sc.order_rank, L.cap,
             at<uint64_t>(ws, L.keys0), at<uint32_t>(ws, L.vals0), at<WsHeader>(ws, L.hdr),
             at<ulonglong2>(ws, L.big_list), L.max_big);
  return hipGetLastError();
}


}  // namespace svr
