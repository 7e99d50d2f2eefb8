// Pixel rendering and its adjoint.
//
// Forward (Sec. 3.1 eq. alpha_blend; Sec. 3.1.2 "Rendering pixels"): one
// workgroup (4 wave64) per 16x16 tile, each wave an 8x8 quadrant, one pixel
// per lane.  The workgroup stages batches of 256 entries of the tile's sorted
// list in LDS (the 64-byte voxel records gathered by voxel id), together with
// a 4-bit mask of the quadrants the voxel's projected rectangle touches; a
// wave skips entries outside its quadrant with a scalar branch.  Per lane: the
// entry's sign pattern must equal the pixel's; the ray-box slab test (Supp.
// A.2 listing "ray_aabb", entry distance > 0) decides a hit; a hit takes K
// midpoint samples (Supp. A.2 eq. K_samp_pts), trilinear corner densities
// (eq. interp), the activation (eq. explin or softplus), optical depth
// x = (l/K) sum act(v_k) and alpha = 1 - exp(-x) (eq. vox_alpha), and is
// composited with the voxel's SH colour.  Transmittance is carried in the
// log domain (tau = sum x), and a lane stops once exp(-tau) < t_stop, i.e.
// a voxel is composited iff the transmittance before it is >= t_stop.  The
// workgroup leaves as soon as all its lanes have stopped.  Saved per pixel:
// tau_final and the list position after the last composited entry.
//
// Backward: the same tiling, walking each pixel's list back to front from its
// saved position and recomputing x and alpha per hit; the transmittance before
// hit i is exp(-(tau_{i+1} - x_i)), so no per-sample state is stored.  With
// S the colour of everything behind hit i seen from just behind it:
//   dL/dc_i = g_rgb T_i alpha_i
//   dL/dx_i = T_{i+1} <g_rgb, c_i - S_i> + g_A T_final
//   dL/dV_m = dL/dx_i (l/K) sum_k act'(v_k) w_m(q_k)    (Supp. A.2 gradient)
// The 11 per-hit gradients are summed over the wave and added with one
// float atomic each.  The pre-process adjoint then maps colour gradients to SH
// coefficients (through the clamp at 0) and scatters corner gradients onto the
// shared grid points.
#include "svr_internal.h"
#include "svr_sh.h"

namespace svr {

constexpr int kBatch = kBlock;

// Sec. 3.1.1 eq. explin:  x for x > 1.1, else exp(x / 1.1 - 1 + ln 1.1)
constexpr float kInv11 = 1.f / 1.1f;
constexpr float kExplinOff = 0.09531017980432486f - 1.f;  // ln(1.1) - 1

template <int ACT>
__device__ __forceinline__ float act_f(float v) {
  if (ACT == SVR_ACT_EXPLIN) return v > 1.1f ? v : __expf(__fmaf_rn(v, kInv11, kExplinOff));
  // softplus, beta = 1: max(v, 0) + log1p(exp(-|v|))
  return fmaxf(v, 0.f) + log1pf(__expf(-fabsf(v)));
}

template <int ACT>
__device__ __forceinline__ float act_df(float v) {
  if (ACT == SVR_ACT_EXPLIN) return v > 1.1f ? 1.f : __expf(__fmaf_rn(v, kInv11, kExplinOff)) * kInv11;
  return 1.f / (1.f + __expf(-v));
}

struct LdsBatch {
  float lx[kBatch], ly[kBatch], lz[kBatch];  // box min - camera centre
  float sz[kBatch], isz[kBatch];             // edge, 1 / edge
  float V[8][kBatch];                        // corner raw densities
  float cr[kBatch], cg[kBatch], cb[kBatch];  // colour
  uint32_t meta[kBatch];                     // sign bits | quadrant mask << 3
  uint32_t vid[kBatch];
};

// Map workgroup -> tile so that each XCD (workgroups are dealt round-robin to
// the 8 XCDs) renders a contiguous block of tiles, which share voxel records
// in that XCD's L2.
__device__ __forceinline__ int xcd_tile(int b, int T) {
  const int per = (T + 7) >> 3;
  return (b & 7) * per + (b >> 3);
}

__device__ __forceinline__ int find_cam_r(const CamSet& cams, int gtile) {
  int c = 0;
  for (int i = 1; i < cams.n; ++i)
    if (gtile >= cams.c[i].tile_off) c = i;
  return c;
}

// stage one entry of the sorted list in LDS
__device__ __forceinline__ void stage_entry(LdsBatch& B, int slot, uint32_t val, int ci, int n_cams,
                                            const VoxRec* __restrict__ rec,
                                            const uint2* __restrict__ rect, int qu0, int qv0) {
  const uint32_t vid = val & kVidMask;
  const int64_t vv = (int64_t)vid * n_cams + ci;
  const VoxRec R = rec[vv];
  const uint2 rc = rect[vv];
  const int u0 = (int)(rc.x & 0xffffu), u1 = (int)(rc.x >> 16);
  const int v0 = (int)(rc.y & 0xffffu), v1 = (int)(rc.y >> 16);
  uint32_t qm = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int a0 = qu0 + (q & 1) * 8, b0 = qv0 + (q >> 1) * 8;
    if (u0 <= a0 + 7 && u1 >= a0 && v0 <= b0 + 7 && v1 >= b0) qm |= 1u << q;
  }
  B.lx[slot] = R.q0.x; B.ly[slot] = R.q0.y; B.lz[slot] = R.q0.z;
  B.sz[slot] = R.q0.w; B.isz[slot] = 1.f / R.q0.w;
  B.V[0][slot] = R.q1.x; B.V[1][slot] = R.q1.y; B.V[2][slot] = R.q1.z; B.V[3][slot] = R.q1.w;
  B.V[4][slot] = R.q2.x; B.V[5][slot] = R.q2.y; B.V[6][slot] = R.q2.z; B.V[7][slot] = R.q2.w;
  B.cr[slot] = R.q3.x; B.cg[slot] = R.q3.y; B.cb[slot] = R.q3.z;
  B.meta[slot] = (val >> kVidBits) | (qm << 3);
  B.vid[slot] = vid;
}

// ray-box slab test against the staged entry j; returns (a, b) and hit flag
__device__ __forceinline__ bool slab(const LdsBatch& B, int j, float idx, float idy, float idz,
                                     float& a, float& b) {
  const float s = B.sz[j];
  const float lx = B.lx[j], ly = B.ly[j], lz = B.lz[j];
  const float t0x = lx * idx, t1x = (lx + s) * idx;
  const float t0y = ly * idy, t1y = (ly + s) * idy;
  const float t0z = lz * idz, t1z = (lz + s) * idz;
  a = fmaxf(fmaxf(fminf(t0x, t1x), fminf(t0y, t1y)), fminf(t0z, t1z));
  b = fminf(fminf(fmaxf(t0x, t1x), fmaxf(t0y, t1y)), fmaxf(t0z, t1z));
  return (a <= b) && (a > 0.f);
}

// trilinear interpolation of the staged corners at local coordinate q
// (corner c = 4x + 2y + z, Supp. A.2 eq. interp)
__device__ __forceinline__ float trilerp(const LdsBatch& B, int j, float qx, float qy, float qz) {
  const float v00 = __fmaf_rn(qz, B.V[1][j] - B.V[0][j], B.V[0][j]);
  const float v01 = __fmaf_rn(qz, B.V[3][j] - B.V[2][j], B.V[2][j]);
  const float v10 = __fmaf_rn(qz, B.V[5][j] - B.V[4][j], B.V[4][j]);
  const float v11 = __fmaf_rn(qz, B.V[7][j] - B.V[6][j], B.V[6][j]);
  const float v0 = __fmaf_rn(qy, v01 - v00, v00);
  const float v1 = __fmaf_rn(qy, v11 - v10, v10);
  return __fmaf_rn(qx, v1 - v0, v0);
}

// ---------------------------------------------------------------------------
// STATS: count, per frame, the (pixel, entry) pairs of matching sign pattern
// the method walks, the ray-box tests this kernel executes after its
// quadrant culling, and the composited hits (into stats[0..2]); no outputs.
template <int K, int ACT, bool STATS>
__global__ __launch_bounds__(kBlock) void k_render_fwd(
    CamSet cams, int T, int n_cams, const uint2* __restrict__ range, const uint32_t* __restrict__ vals,
    const VoxRec* __restrict__ rec, const uint2* __restrict__ rect, float t_stop,
    float4* __restrict__ rgba, float* __restrict__ px_tau, uint32_t* __restrict__ px_last,
    unsigned long long* __restrict__ stats) {
  __shared__ LdsBatch B;
  const int g = xcd_tile(blockIdx.x, T);
  if (g >= T) return;
  const int ci = find_cam_r(cams, g);
  const DevCam& c = cams.c[ci];
  const int tl = g - c.tile_off;
  const int tx = tl % c.ntx, ty = tl / c.ntx;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int qu0 = tx * kTile, qv0 = ty * kTile;
  const int u = qu0 + (w & 1) * 8 + (lane & 7);
  const int v = qv0 + (w >> 1) * 8 + (lane >> 3);
  const bool inside = u < c.W && v < c.H;
  float dx, dy, dz;
  pixel_dir(c, u, v, dx, dy, dz);
  const uint32_t spat = (uint32_t)sign_bits(dx, dy, dz);
  const float rn = rsqrtf(dx * dx + dy * dy + dz * dz);
  dx *= rn; dy *= rn; dz *= rn;
  const float idx = 1.f / dx, idy = 1.f / dy, idz = 1.f / dz;

  const uint2 rg = range[g];
  const uint32_t start = rg.x, end = rg.y;
  float tau = 0.f, Tr = 1.f, C0 = 0.f, C1 = 0.f, C2 = 0.f;
  uint32_t last = start;
  bool done = !inside;
  uint32_t n_pairs = 0, n_tests = 0, n_hits = 0;
  for (uint32_t b0 = start; b0 < end; b0 += kBatch) {
    const uint32_t i = b0 + tid;
    if (i < end) stage_entry(B, tid, vals[i], ci, n_cams, rec, rect, qu0, qv0);
    __syncthreads();
    const int n = (int)min((uint32_t)kBatch, end - b0);
    for (int j = 0; j < n; ++j) {
      const uint32_t meta = __builtin_amdgcn_readfirstlane(B.meta[j]);
      if (STATS && !done && (meta & 7u) == spat) ++n_pairs;
      if (!((meta >> (3 + w)) & 1u)) continue;
      if (done || (meta & 7u) != spat) continue;
      float a, bb;
      if (STATS) ++n_tests;
      if (!slab(B, j, idx, idy, idz, a, bb)) continue;
      if (STATS) ++n_hits;
      const float l = bb - a;
      const float lx = B.lx[j], ly = B.ly[j], lz = B.lz[j], is = B.isz[j];
      float x = 0.f;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const float t = __fmaf_rn(((float)k + 0.5f) * (1.f / K), l, a);
        const float qx = (t * dx - lx) * is, qy = (t * dy - ly) * is, qz = (t * dz - lz) * is;
        x += act_f<ACT>(trilerp(B, j, qx, qy, qz));
      }
      x *= l * (1.f / K);
      const float wgt = Tr * (1.f - __expf(-x));
      C0 = __fmaf_rn(wgt, B.cr[j], C0);
      C1 = __fmaf_rn(wgt, B.cg[j], C1);
      C2 = __fmaf_rn(wgt, B.cb[j], C2);
      tau += x;
      Tr = __expf(-tau);
      last = b0 + (uint32_t)j + 1u;
      if (Tr < t_stop) done = true;
    }
    if (__syncthreads_and(done)) break;
  }
  if (STATS) {
    unsigned long long a0 = n_pairs, a1 = n_tests, a2 = n_hits;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      a0 += __shfl_xor(a0, o, 64);
      a1 += __shfl_xor(a1, o, 64);
      a2 += __shfl_xor(a2, o, 64);
    }
    if (lane == 0) {
      atomicAdd(stats + 0, a0);
      atomicAdd(stats + 1, a1);
      atomicAdd(stats + 2, a2);
    }
    return;
  }
  if (inside) {
    const int64_t p = c.pix_off + (int64_t)v * c.W + u;
    rgba[p] = make_float4(C0, C1, C2, 1.f - Tr);
    px_tau[p] = tau;
    px_last[p] = last;
  }
}

// ---------------------------------------------------------------------------
__device__ __forceinline__ float wave_sum(float x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

template <int K, int ACT>
__global__ __launch_bounds__(kBlock) void k_render_bwd(
    CamSet cams, int T, int n_cams, const uint2* __restrict__ range, const uint32_t* __restrict__ vals,
    const VoxRec* __restrict__ rec, const uint2* __restrict__ rect,
    const float* __restrict__ px_tau, const uint32_t* __restrict__ px_last,
    const float4* __restrict__ grad_rgba, float* __restrict__ g_corner, float* __restrict__ g_rgb) {
  __shared__ LdsBatch B;
  __shared__ uint32_t s_lmax;
  const int g = xcd_tile(blockIdx.x, T);
  if (g >= T) return;
  const int ci = find_cam_r(cams, g);
  const DevCam& c = cams.c[ci];
  const int tl = g - c.tile_off;
  const int tx = tl % c.ntx, ty = tl / c.ntx;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int qu0 = tx * kTile, qv0 = ty * kTile;
  const int u = qu0 + (w & 1) * 8 + (lane & 7);
  const int v = qv0 + (w >> 1) * 8 + (lane >> 3);
  const bool inside = u < c.W && v < c.H;
  float dx, dy, dz;
  pixel_dir(c, u, v, dx, dy, dz);
  const uint32_t spat = (uint32_t)sign_bits(dx, dy, dz);
  const float rn = rsqrtf(dx * dx + dy * dy + dz * dz);
  dx *= rn; dy *= rn; dz *= rn;
  const float idx = 1.f / dx, idy = 1.f / dy, idz = 1.f / dz;

  const uint2 rg = range[g];
  const uint32_t start = rg.x;
  float tau = 0.f, gr = 0.f, gg = 0.f, gb = 0.f, ga = 0.f;
  uint32_t last = start;
  if (inside) {
    const int64_t p = c.pix_off + (int64_t)v * c.W + u;
    tau = px_tau[p];
    last = px_last[p];
    const float4 gq = grad_rgba[p];
    gr = gq.x; gg = gq.y; gb = gq.z; ga = gq.w;
  }
  const float Tfin = __expf(-tau);
  float S0 = 0.f, S1 = 0.f, S2 = 0.f;
  if (tid == 0) s_lmax = start;
  __syncthreads();
  if (last > start) atomicMax(&s_lmax, last);
  __syncthreads();
  const uint32_t lmax = s_lmax;

  uint32_t bend = lmax;
  while (bend > start) {
    const uint32_t b0 = bend - min((uint32_t)kBatch, bend - start);
    const int n = (int)(bend - b0);
    bend = b0;
    if (tid < n) stage_entry(B, tid, vals[b0 + tid], ci, n_cams, rec, rect, qu0, qv0);
    __syncthreads();
    for (int j = n - 1; j >= 0; --j) {
      const uint32_t meta = __builtin_amdgcn_readfirstlane(B.meta[j]);
      if (!((meta >> (3 + w)) & 1u)) continue;
      float a = 0.f, bb = 0.f;
      bool hit = (b0 + (uint32_t)j < last) && ((meta & 7u) == spat);
      if (hit) hit = slab(B, j, idx, idy, idz, a, bb);
      if (__ballot(hit) == 0ull) continue;
      float gV[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      float gc0 = 0.f, gc1 = 0.f, gc2 = 0.f;
      if (hit) {
        const float l = bb - a;
        const float lx = B.lx[j], ly = B.ly[j], lz = B.lz[j], is = B.isz[j];
        float x = 0.f;
        float dw[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};  // sum_k act'(v_k) w_m(q_k)
#pragma unroll
        for (int k = 0; k < K; ++k) {
          const float t = __fmaf_rn(((float)k + 0.5f) * (1.f / K), l, a);
          const float qx = (t * dx - lx) * is, qy = (t * dy - ly) * is, qz = (t * dz - lz) * is;
          const float vk = trilerp(B, j, qx, qy, qz);
          x += act_f<ACT>(vk);
          const float dk = act_df<ACT>(vk);
          const float px = 1.f - qx, py = 1.f - qy, pz = 1.f - qz;
          const float a00 = dk * px * py, a01 = dk * px * qy, a10 = dk * qx * py, a11 = dk * qx * qy;
          dw[0] = __fmaf_rn(a00, pz, dw[0]); dw[1] = __fmaf_rn(a00, qz, dw[1]);
          dw[2] = __fmaf_rn(a01, pz, dw[2]); dw[3] = __fmaf_rn(a01, qz, dw[3]);
          dw[4] = __fmaf_rn(a10, pz, dw[4]); dw[5] = __fmaf_rn(a10, qz, dw[5]);
          dw[6] = __fmaf_rn(a11, pz, dw[6]); dw[7] = __fmaf_rn(a11, qz, dw[7]);
        }
        const float lK = l * (1.f / K);
        x *= lK;
        const float e = __expf(-x);
        const float alpha = 1.f - e;
        const float Tnext = __expf(-tau);
        tau -= x;
        const float Ti = __expf(-tau);
        const float cr = B.cr[j], cg = B.cg[j], cb = B.cb[j];
        const float wgt = Ti * alpha;
        gc0 = gr * wgt; gc1 = gg * wgt; gc2 = gb * wgt;
        const float dLdx = Tnext * (gr * (cr - S0) + gg * (cg - S1) + gb * (cb - S2)) + ga * Tfin;
        S0 = __fmaf_rn(alpha, cr - S0, S0);
        S1 = __fmaf_rn(alpha, cg - S1, S1);
        S2 = __fmaf_rn(alpha, cb - S2, S2);
        const float f = dLdx * lK;
#pragma unroll
        for (int m = 0; m < 8; ++m) gV[m] = f * dw[m];
      }
#pragma unroll
      for (int m = 0; m < 8; ++m) gV[m] = wave_sum(gV[m]);
      gc0 = wave_sum(gc0); gc1 = wave_sum(gc1); gc2 = wave_sum(gc2);
      if (lane == 0) {
        const uint32_t vid = B.vid[j];
        float* gcp = g_corner + (int64_t)vid * 8;
#pragma unroll
        for (int m = 0; m < 8; ++m) unsafeAtomicAdd(gcp + m, gV[m]);
        float* grp = g_rgb + ((int64_t)vid * n_cams + ci) * 3;
        unsafeAtomicAdd(grp + 0, gc0);
        unsafeAtomicAdd(grp + 1, gc1);
        unsafeAtomicAdd(grp + 2, gc2);
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
template <int D>
__global__ __launch_bounds__(kBlock) void k_sh_bwd(
    int64_t N, int n_cams, CamSet cams, const float* __restrict__ center,
    const int32_t* __restrict__ vox_grid, const uint32_t* __restrict__ count,
    const VoxRec* __restrict__ rec, const float* __restrict__ g_rgb,
    const float* __restrict__ g_corner, float* __restrict__ grad_grid, float* __restrict__ grad_sh) {
  constexpr int NB = (D + 1) * (D + 1);
  const int64_t vid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (vid >= N) return;
  if (grad_sh) {
    float acc[NB][3];
#pragma unroll
    for (int j = 0; j < NB; ++j) acc[j][0] = acc[j][1] = acc[j][2] = 0.f;
    for (int ci = 0; ci < n_cams; ++ci) {
      const int64_t vv = vid * n_cams + ci;
      if (count[vv] == 0) continue;
      const DevCam& c = cams.c[ci];
      const uint32_t bits = __float_as_uint(rec[vv].q3.w);
      float g3[3];
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) g3[ch] = ((bits >> ch) & 1u) ? g_rgb[vv * 3 + ch] : 0.f;
      const float rx = center[vid] - c.o[0], ry = center[N + vid] - c.o[1],
                  rz = center[2 * N + vid] - c.o[2];
      const float rn = rsqrtf(rx * rx + ry * ry + rz * rz);
      float Y[16];
      sh_basis<D>(rx * rn, ry * rn, rz * rn, Y);
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        acc[j][0] = __fmaf_rn(g3[0], Y[j], acc[j][0]);
        acc[j][1] = __fmaf_rn(g3[1], Y[j], acc[j][1]);
        acc[j][2] = __fmaf_rn(g3[2], Y[j], acc[j][2]);
      }
    }
    float* o = grad_sh + vid * (3 * NB);
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      o[3 * j + 0] = acc[j][0];
      o[3 * j + 1] = acc[j][1];
      o[3 * j + 2] = acc[j][2];
    }
  }
  if (grad_grid) {
    const float4* gc = reinterpret_cast<const float4*>(g_corner + vid * 8);
    const float4 ga = gc[0], gb = gc[1];
    const float gv[8] = {ga.x, ga.y, ga.z, ga.w, gb.x, gb.y, gb.z, gb.w};
    const int4* vg = reinterpret_cast<const int4*>(vox_grid + vid * 8);
    const int4 ia = vg[0], ib = vg[1];
    const int idxs[8] = {ia.x, ia.y, ia.z, ia.w, ib.x, ib.y, ib.z, ib.w};
#pragma unroll
    for (int m = 0; m < 8; ++m)
      if (gv[m] != 0.f) unsafeAtomicAdd(grad_grid + idxs[m], gv[m]);
  }
}

// ---------------------------------------------------------------------------
template <int K, int ACT>
static void launch_fwd_t(dim3 grid, hipStream_t s, const CamSet& cams, const Layout& L, void* ws,
                         const uint32_t* vals, float t_stop, float* rgba) {
  SVR_LAUNCH("render_fwd", (k_render_fwd<K, ACT, false>), grid, dim3(kBlock), 0, s, cams, L.T,
             L.n_cams, at<uint2>(ws, L.tile_range), vals, at<VoxRec>(ws, L.rec),
             at<uint2>(ws, L.rect), t_stop, reinterpret_cast<float4*>(rgba),
             at<float>(ws, L.px_tau), at<uint32_t>(ws, L.px_last), nullptr);
}

template <int K, int ACT>
static void launch_stats_t(dim3 grid, hipStream_t s, const CamSet& cams, const Layout& L, void* ws,
                           const uint32_t* vals, float t_stop) {
  SVR_LAUNCH("render_stats", (k_render_fwd<K, ACT, true>), grid, dim3(kBlock), 0, s, cams, L.T,
             L.n_cams, at<uint2>(ws, L.tile_range), vals, at<VoxRec>(ws, L.rec),
             at<uint2>(ws, L.rect), t_stop, nullptr, nullptr, nullptr,
             at<WsHeader>(ws, L.hdr)->stats);
}

template <int K, int ACT>
static void launch_bwd_t(dim3 grid, hipStream_t s, const CamSet& cams, const Layout& L, void* ws,
                         const uint32_t* vals, const float* grad_rgba) {
  SVR_LAUNCH("render_bwd", (k_render_bwd<K, ACT>), grid, dim3(kBlock), 0, s, cams, L.T, L.n_cams,
                     at<uint2>(ws, L.tile_range), vals, at<VoxRec>(ws, L.rec), at<uint2>(ws, L.rect),
                     at<float>(ws, L.px_tau), at<uint32_t>(ws, L.px_last),
                     reinterpret_cast<const float4*>(grad_rgba), at<float>(ws, L.g_corner),
                     at<float>(ws, L.g_rgb));
}

#define SVR_DISPATCH_K(FN, ACT, ...)             \
  switch (o.K) {                                 \
    case 1: FN<1, ACT>(__VA_ARGS__); break;      \
    case 2: FN<2, ACT>(__VA_ARGS__); break;      \
    case 3: FN<3, ACT>(__VA_ARGS__); break;      \
    case 4: FN<4, ACT>(__VA_ARGS__); break;      \
    case 5: FN<5, ACT>(__VA_ARGS__); break;      \
    case 6: FN<6, ACT>(__VA_ARGS__); break;      \
    case 7: FN<7, ACT>(__VA_ARGS__); break;      \
    default: FN<8, ACT>(__VA_ARGS__); break;     \
  }

static dim3 render_grid(int T) { return dim3((unsigned)(((T + 7) >> 3) << 3)); }

hipError_t launch_render_fwd(const svr_scene& sc, const CamSet& cams, const svr_opts& o,
                             const Layout& L, void* ws, const uint32_t* vals, float* rgba,
                             hipStream_t s) {
  (void)sc;
  if (L.T == 0) return hipSuccess;
  const dim3 grid = render_grid(L.T);
  if (o.activation == SVR_ACT_SOFTPLUS) {
    SVR_DISPATCH_K(launch_fwd_t, SVR_ACT_SOFTPLUS, grid, s, cams, L, ws, vals, o.t_stop, rgba)
  } else {
    SVR_DISPATCH_K(launch_fwd_t, SVR_ACT_EXPLIN, grid, s, cams, L, ws, vals, o.t_stop, rgba)
  }
  return hipGetLastError();
}

hipError_t launch_render_stats(const svr_scene& sc, const CamSet& cams, const svr_opts& o,
                               const Layout& L, void* ws, const uint32_t* vals, hipStream_t s) {
  (void)sc;
  hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t*>(at<WsHeader>(ws, L.hdr)->stats), 0u,
                                 6, s);
  if (e != hipSuccess) return e;
  if (L.T == 0) return hipSuccess;
  const dim3 grid = render_grid(L.T);
  if (o.activation == SVR_ACT_SOFTPLUS) {
    SVR_DISPATCH_K(launch_stats_t, SVR_ACT_SOFTPLUS, grid, s, cams, L, ws, vals, o.t_stop)
  } else {
    SVR_DISPATCH_K(launch_stats_t, SVR_ACT_EXPLIN, grid, s, cams, L, ws, vals, o.t_stop)
  }
  return hipGetLastError();
}

hipError_t launch_render_bwd(const svr_scene& sc, const CamSet& cams, const svr_opts& o,
                             const Layout& L, void* ws, const uint32_t* vals,
                             const float* grad_rgba, hipStream_t s) {
  (void)sc;
  hipError_t e = launch_fill_u32(at<uint32_t>(ws, L.g_corner), 0u, L.N * 8, s);
  if (e != hipSuccess) return e;
  e = launch_fill_u32(at<uint32_t>(ws, L.g_rgb), 0u, L.NV * 3, s);
  if (e != hipSuccess) return e;
  if (L.T == 0) return hipSuccess;
  const dim3 grid = render_grid(L.T);
  if (o.activation == SVR_ACT_SOFTPLUS) {
    SVR_DISPATCH_K(launch_bwd_t, SVR_ACT_SOFTPLUS, grid, s, cams, L, ws, vals, grad_rgba)
  } else {
    SVR_DISPATCH_K(launch_bwd_t, SVR_ACT_EXPLIN, grid, s, cams, L, ws, vals, grad_rgba)
  }
  return hipGetLastError();
}

hipError_t launch_sh_bwd(const svr_scene& sc, const CamSet& cams, const Layout& L, void* ws,
                         float* grad_grid, float* grad_sh, hipStream_t s) {
  if (grad_grid) {
    hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t*>(grad_grid), 0u, sc.n_grid, s);
    if (e != hipSuccess) return e;
  }
  if (L.N == 0) return hipSuccess;
  const dim3 grid((unsigned)((L.N + kBlock - 1) / kBlock));
#define SVR_SHB(D)                                                                             \
  SVR_LAUNCH("sh_bwd", k_sh_bwd<D>, grid, dim3(kBlock), 0, s, L.N, L.n_cams, cams, sc.center,   \
                     sc.vox_grid, at<uint32_t>(ws, L.count), at<VoxRec>(ws, L.rec),            \
                     at<float>(ws, L.g_rgb), at<float>(ws, L.g_corner), grad_grid, grad_sh)
  switch (sc.sh_degree) {
    case 0: SVR_SHB(0); break;
    case 1: SVR_SHB(1); break;
    case 2: SVR_SHB(2); break;
    default: SVR_SHB(3); break;
  }
#undef SVR_SHB
  return hipGetLastError();
}

}  // namespace svr
