// Pixel rendering and its adjoint.
//
// Forward (Sec. 3.1 eq. alpha_blend; Sec. 3.1.2 "Rendering pixels"): one
// workgroup per TSxTS tile (TS = 8, 16 or 32: 1, 4 or 16 wave64), each wave an
// 8x8 pixel block, one pixel per lane.  The workgroup stages batches of up to
// 256 entries of the tile's sorted list in LDS (the 64-byte voxel records
// gathered by voxel id), together with a mask of the 8x8 blocks the voxel's
// projected rectangle touches; a wave skips entries outside its block with a
// scalar branch.  Per lane: the entry's sign pattern must equal the pixel's;
// the ray-box slab test (Supp. A.2 listing "ray_aabb", entry distance > 0)
// decides a hit; a hit takes K midpoint samples (Supp. A.2 eq. K_samp_pts),
// trilinear corner densities (eq. interp), the activation (eq. explin or
// softplus), optical depth x = (l/K) sum act(v_k) and alpha = 1 - exp(-x)
// (eq. vox_alpha), and is composited with the voxel's SH colour.
// Transmittance is carried in the log domain (tau = sum x), and a lane stops
// once exp(-tau) < t_stop, i.e. a voxel is composited iff the transmittance
// before it is >= t_stop.  A tile ends as soon as all its lanes have stopped.
// Saved per pixel: tau_final and the list position after the last composited
// entry.
//
// Backward: the same tiling, walking each pixel's list back to front from its
// saved position and recomputing x and alpha per hit; the transmittance before
// hit i is exp(-(tau_{i+1} - x_i)), so no per-sample state is stored.  With
// U_{i+1} = sum_{j>i} T_j alpha_j c_j the colour composited after hit i:
//   dL/dc_i = g_rgb T_i alpha_i
//   dL/dx_i = <g_rgb, T_{i+1} c_i - U_{i+1}> + g_A T_final
//   dL/dV_m = dL/dx_i (l/K) sum_k act'(v_k) w_m(q_k)    (Supp. A.2 gradient)
// and U_i = U_{i+1} + T_i alpha_i c_i.  The 11 per-hit gradients (12 with the
// subdivision priority |alpha_i dL/dalpha_i| of Sec. 3.2.2) are summed over
// the wave and added with one float atomic per value.  A tile with more
// than kBwdChunk entries is split into chunks of that many entries, one
// workgroup each: the forward saves, per pixel, tau and the colour still to
// come at every chunk boundary it passes, which is all a chunk's reverse walk
// needs to start.  The pre-process adjoint then maps colour gradients to SH
// coefficients (through the clamp at 0) and gathers corner gradients onto the
// shared grid points.
//
// Tile scheduling: tiles are rendered in the order the sort stage leaves in
// the workspace, heaviest (most entries) first, because the per-tile work is
// skewed (a few silhouette tiles hold 10-20x the mean) and a heavy tile
// started last would set the kernel's length.  Either one workgroup per
// position of that order, or a persistent grid whose workgroups take the next
// position from one counter.
#include <type_traits>

#include "svr_internal.h"
#include "svr_sh.h"

namespace svr {

// backward walk: entries grouped by disjoint pixel sets (true) or one entry
// at a time (false)
constexpr bool kGroupedBwd = true;

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

// alpha = 1 - exp(-x) (eq. vox_alpha).  For small optical depth the
// difference cancels in fp32 (exp(-x) rounds to 1 for x < 6e-8), so below
// x = 2^-7 the Taylor series x (1 - x/2 + x^2/6) is used instead; its
// truncation error x^3/24 relative is below 1e-7 there.
__device__ __forceinline__ float alpha_of(float x) {
  const float taylor = x * __fmaf_rn(x, __fmaf_rn(x, 1.f / 6.f, -0.5f), 1.f);
  return x < 0.0078125f ? taylor : 1.f - __expf(-x);
}


template <int TS>
struct TileGeom {
  static constexpr int kThreads = TS * TS;
  static constexpr int kWaves = kThreads / 64;
  static constexpr int kBpr = TS / 8;  // 8x8 blocks per tile row
  static constexpr int kBatch = kThreads < 256 ? kThreads : 256;
};

template <int NB>
struct LdsBatch {
  double lo[3][NB];                    // box min - camera centre (fp64)
  float4 col[NB];                      // colour rgb, voxel id (bits) in w
  float edge[NB];                      // box edge (box max = min + edge)
  float isz[NB];                       // 1 / edge
  float V[8][NB];                      // trilinear coefficients of the corner raw densities
  uint32_t meta[NB];                   // sign bits | block mask << 3
  uint32_t rx[NB], ry[NB];             // pixel rectangle: u0 | u1 << 16, v0 | v1 << 16
};

// arguments shared by the render kernels
struct RenderArgs {
  CamSet cams;
  int T, n_cams, K, persistent;
  float t_stop;
  const uint2* range;
  const uint32_t* vals;
  const VoxRec* rec;
  const uint2* rect;
  float4* rgba;
  float* px_tau;
  uint32_t* px_last;
  unsigned long long* stats;
  const float4* grad_rgba;
  float* g_corner;
  float* g_rgb;
  uint32_t* work;  // persistent mode: work[0] next chunk item, work[1] next render position
  const uint32_t* order;  // render order of the tiles (heaviest first)
  // backward chunks of heavy tiles
  const uint32_t* split_base;   // per tile: first item / checkpoint slot, or kNoSplit
  const uint2* split_items;     // (tile, chunk) for every chunk but a tile's last
  const uint32_t* split_count;  // number of items
  float4* ckpt;                 // per slot and pixel: (tau, suffix colour) at the chunk's end
  int max_split, split_wgs;
  uint32_t* max_weight;         // training statistics (bit patterns of non-negative floats)
  float* priority;
  // depth and normal images (aux kernels)
  float* depth;
  float* normal;
  const float* grad_depth;
  const float* grad_normal;
  float4* ckpt_aux;             // per slot and pixel: (depth, normal) still to come
  float* g_nrm;                 // per voxel dL/dn
  int aux;
};

// next position in the render order for a persistent workgroup (-1: none left)
__device__ __forceinline__ int next_tile(uint32_t* work, int T) {
  const uint32_t p = atomicAdd(work, 1u);
  return p < (uint32_t)T ? (int)p : -1;
}

__device__ __forceinline__ int find_cam_r(const CamSet& cams, int gtile) {
  int c = 0;
  for (int i = 1; i < cams.n; ++i)
    if (gtile >= cams.c[i].tile_off) c = i;
  return c;
}

// stage one entry of the sorted list in LDS
template <int TS, int NB>
__device__ __forceinline__ void stage_entry(LdsBatch<NB>& B, int slot, uint32_t val, int ci,
                                            int n_cams, const DevCam& c,
                                            const VoxRec* __restrict__ rec,
                                            const uint2* __restrict__ rect, int qu0, int qv0) {
  using G = TileGeom<TS>;
  const uint32_t vid = val & kVidMask;
  const int64_t vv = (int64_t)vid * n_cams + ci;
  const VoxRec R = rec[vv];
  const uint2 rc = rect[vv];
  const int u0 = (int)(rc.x & 0xffffu), u1 = (int)(rc.x >> 16);
  const int v0 = (int)(rc.y & 0xffffu), v1 = (int)(rc.y >> 16);
  uint32_t qm = 0;
#pragma unroll
  for (int q = 0; q < G::kWaves; ++q) {
    const int a0 = qu0 + (q % G::kBpr) * 8, b0 = qv0 + (q / G::kBpr) * 8;
    if (u0 <= a0 + 7 && u1 >= a0 && v0 <= b0 + 7 && v1 >= b0) qm |= 1u << q;
  }
  const double h = 0.5 * (double)R.q0.w;
  const double lx = ((double)R.q0.x - h) - c.od[0];
  const double ly = ((double)R.q0.y - h) - c.od[1];
  const double lz = ((double)R.q0.z - h) - c.od[2];
  B.lo[0][slot] = lx;
  B.lo[1][slot] = ly;
  B.lo[2][slot] = lz;
  B.edge[slot] = R.q0.w;
  B.isz[slot] = 1.f / R.q0.w;
  // the field over the voxel as c0 + c1 x + c2 y + c3 z + c4 xy + c5 xz +
  // c6 yz + c7 xyz (corner c = 4x + 2y + z), so that an interpolation is 7
  // fused multiply-adds
  const float d0 = R.q1.x, d1 = R.q1.y, d2 = R.q1.z, d3 = R.q1.w;
  const float d4 = R.q2.x, d5 = R.q2.y, d6 = R.q2.z, d7 = R.q2.w;
  B.V[0][slot] = d0;
  B.V[1][slot] = d4 - d0;
  B.V[2][slot] = d2 - d0;
  B.V[3][slot] = d1 - d0;
  B.V[4][slot] = (d6 - d4) - (d2 - d0);
  B.V[5][slot] = (d5 - d4) - (d1 - d0);
  B.V[6][slot] = (d3 - d2) - (d1 - d0);
  B.V[7][slot] = ((d7 - d6) - (d5 - d4)) - ((d3 - d2) - (d1 - d0));
  B.col[slot] = make_float4(R.q3.x, R.q3.y, R.q3.z, __uint_as_float(vid));
  B.meta[slot] = (val >> kVidBits) | (qm << 3);
  B.rx[slot] = rc.x;
  B.ry[slot] = rc.y;
}

// Ray-box slab test (Supp. A.2 listing "ray_aabb") against staged entry j, in
// fp64: entry/exit distances a <= b, hit iff a <= b and a > 0.
template <int NB>
__device__ __forceinline__ bool slab(const LdsBatch<NB>& B, int j, double idx, double idy,
                                     double idz, double& a, double& b) {
  const double e = (double)B.edge[j];
  const double lx = B.lo[0][j], ly = B.lo[1][j], lz = B.lo[2][j];
  const double t0x = lx * idx, t1x = (lx + e) * idx;
  const double t0y = ly * idy, t1y = (ly + e) * idy;
  const double t0z = lz * idz, t1z = (lz + e) * idz;
  a = fmax(fmax(fmin(t0x, t1x), fmin(t0y, t1y)), fmin(t0z, t1z));
  b = fmin(fmin(fmax(t0x, t1x), fmax(t0y, t1y)), fmax(t0z, t1z));
  return (a <= b) && (a > 0.0);
}

// local voxel coordinate of the point at distance t on the ray (Supp. A.2
// eq. K_samp_pts): q = (o + t d - box min) / edge, in fp64 then rounded
template <int NB>
__device__ __forceinline__ void local_coord(const LdsBatch<NB>& B, int j, double t, double dx,
                                            double dy, double dz, float& qx, float& qy,
                                            float& qz) {
  const float is = B.isz[j];
  qx = (float)fma(t, dx, -B.lo[0][j]) * is;
  qy = (float)fma(t, dy, -B.lo[1][j]) * is;
  qz = (float)fma(t, dz, -B.lo[2][j]) * is;
}

// trilinear interpolation of the staged field at local coordinate q
// (Supp. A.2 eq. interp), from its coefficients
template <int NB>
__device__ __forceinline__ float trilerp(const LdsBatch<NB>& B, int j, float qx, float qy,
                                         float qz) {
  const float a = __fmaf_rn(B.V[3][j], qz, B.V[0][j]);  // c0 + c3 z
  const float b = __fmaf_rn(B.V[6][j], qz, B.V[2][j]);  // c2 + c6 z
  const float c = __fmaf_rn(B.V[5][j], qz, B.V[1][j]);  // c1 + c5 z
  const float d = __fmaf_rn(B.V[7][j], qz, B.V[4][j]);  // c4 + c7 z
  return __fmaf_rn(__fmaf_rn(d, qy, c), qx, __fmaf_rn(b, qy, a));
}

struct PixelRay {
  int u, v;
  bool inside;
  uint32_t spat;         // ray sign bits (from the fp32 direction, as the tile masks)
  double dx, dy, dz;     // unit direction, fp64
  double idx, idy, idz;  // its reciprocal
};

template <int TS>
__device__ __forceinline__ PixelRay make_ray(const DevCam& c, int qu0, int qv0, int w, int lane) {
  using G = TileGeom<TS>;
  PixelRay r;
  r.u = qu0 + (w % G::kBpr) * 8 + (lane & 7);
  r.v = qv0 + (w / G::kBpr) * 8 + (lane >> 3);
  r.inside = r.u < c.W && r.v < c.H;
  float fx, fy, fz;
  pixel_dir(c, r.u, r.v, fx, fy, fz);
  r.spat = (uint32_t)sign_bits(fx, fy, fz);
  pixel_dir_f64(c, r.u, r.v, r.dx, r.dy, r.dz);
  r.idx = 1.0 / r.dx;
  r.idy = 1.0 / r.dy;
  r.idz = 1.0 / r.dz;
  return r;
}

// optical depth of staged entry j on the ray over [a, b]; with DW also the
// sums sum_k act'(v_k) w_m(q_k) of the 8 corner weights
template <int KT, int ACT, bool DW, int NB>
__device__ __forceinline__ float segment_x(const LdsBatch<NB>& B, int j, double dx, double dy,
                                           double dz, double a, double lseg, int Krt, float* dw) {
  const int K = KT > 0 ? KT : Krt;
  const double step = 1.0 / (double)K;
  float x = 0.f;
#pragma unroll
  for (int k = 0; k < (KT > 0 ? KT : SVR_MAX_K); ++k) {
    if (KT == 0 && k >= K) break;
    const double t = fma(((double)k + 0.5) * step, lseg, a);
    float qx, qy, qz;
    local_coord(B, j, t, dx, dy, dz, qx, qy, qz);
    const float vk = trilerp(B, j, qx, qy, qz);
    x += act_f<ACT>(vk);
    if (DW) {
      const float dk = act_df<ACT>(vk);
      const float px = 1.f - qx, py = 1.f - qy, pz = 1.f - qz;
      const float a00 = dk * px * py, a01 = dk * px * qy, a10 = dk * qx * py, a11 = dk * qx * qy;
      dw[0] = __fmaf_rn(a00, pz, dw[0]); dw[1] = __fmaf_rn(a00, qz, dw[1]);
      dw[2] = __fmaf_rn(a01, pz, dw[2]); dw[3] = __fmaf_rn(a01, qz, dw[3]);
      dw[4] = __fmaf_rn(a10, pz, dw[4]); dw[5] = __fmaf_rn(a10, qz, dw[5]);
      dw[6] = __fmaf_rn(a11, pz, dw[6]); dw[7] = __fmaf_rn(a11, qz, dw[7]);
    }
  }
  return x * ((float)lseg / (float)K);
}

// Backward form of segment_x for a compile-time K: the optical depth, and
// per sample its local coordinate and act'(v_k), so that the corner
// gradients f sum_k act'(v_k) w_m(q_k) can be formed once f = dL/dx (l/K) is
// known, with f folded into each sample's factor
template <int KT, int ACT, int NB>
__device__ __forceinline__ float segment_samples(const LdsBatch<NB>& B, int j, double dx, double dy,
                                                 double dz, double a, double lseg, float (&q)[KT][3],
                                                 float (&dk)[KT]) {
  const double step = 1.0 / (double)KT;
  float x = 0.f;
#pragma unroll
  for (int k = 0; k < KT; ++k) {
    const double t = fma(((double)k + 0.5) * step, lseg, a);
    local_coord(B, j, t, dx, dy, dz, q[k][0], q[k][1], q[k][2]);
    const float vk = trilerp(B, j, q[k][0], q[k][1], q[k][2]);
    x += act_f<ACT>(vk);
    dk[k] = act_df<ACT>(vk);
  }
  return x * ((float)lseg / (float)KT);
}

// g[m] = sum_k f dk_k w_m(q_k) for the 8 corners (trilinear weights w_m)
template <int KT>
__device__ __forceinline__ void corner_grads(const float (&q)[KT][3], const float (&dk)[KT], float f,
                                             float (&g)[16]) {
#pragma unroll
  for (int m = 0; m < 8; ++m) g[m] = 0.f;
#pragma unroll
  for (int k = 0; k < KT; ++k) {
    const float fk = f * dk[k];
    const float qx = q[k][0], qy = q[k][1], qz = q[k][2];
    const float px = 1.f - qx, py = 1.f - qy, pz = 1.f - qz;
    const float bx0 = fk * px, bx1 = fk * qx;
    const float a00 = bx0 * py, a01 = bx0 * qy, a10 = bx1 * py, a11 = bx1 * qy;
    g[0] = __fmaf_rn(a00, pz, g[0]); g[1] = __fmaf_rn(a00, qz, g[1]);
    g[2] = __fmaf_rn(a01, pz, g[2]); g[3] = __fmaf_rn(a01, qz, g[3]);
    g[4] = __fmaf_rn(a10, pz, g[4]); g[5] = __fmaf_rn(a10, qz, g[5]);
    g[6] = __fmaf_rn(a11, pz, g[6]); g[7] = __fmaf_rn(a11, qz, g[7]);
  }
}

// Voxel normal (Sec. 3.1.1 "Voxel normal"; Supp. details of voxel normal):
// the gradient of the trilinear raw density at the voxel centre,
//   g = 0.25 ((V_1jk summed) - (V_0jk summed), ...) for x, y, z,
// normalised (zero when g = 0).  Corner c = 4x + 2y + z.
__device__ __forceinline__ void centre_gradient(const float V[8], float g[3]) {
  g[0] = 0.25f * ((V[4] + V[5] + V[6] + V[7]) - (V[0] + V[1] + V[2] + V[3]));
  g[1] = 0.25f * ((V[2] + V[3] + V[6] + V[7]) - (V[0] + V[1] + V[4] + V[5]));
  g[2] = 0.25f * ((V[1] + V[3] + V[5] + V[7]) - (V[0] + V[2] + V[4] + V[6]));
}

template <int NB>
__device__ __forceinline__ void staged_normal(const LdsBatch<NB>& B, int j, float n[3]) {
  // the centre gradient from the staged coefficients (the derivative of the
  // field at q = (1/2, 1/2, 1/2))
  float g[3];
  g[0] = B.V[1][j] + 0.5f * (B.V[4][j] + B.V[5][j]) + 0.25f * B.V[7][j];
  g[1] = B.V[2][j] + 0.5f * (B.V[4][j] + B.V[6][j]) + 0.25f * B.V[7][j];
  g[2] = B.V[3][j] + 0.5f * (B.V[5][j] + B.V[6][j]) + 0.25f * B.V[7][j];
  const float g2 = g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
  const float r = g2 > 0.f ? rsqrtf(g2) : 0.f;
  n[0] = g[0] * r; n[1] = g[1] * r; n[2] = g[2] * r;
}

// optical depth x of staged entry j (as segment_x) and its local depth
// (Supp. details of voxel depth): the K samples composited with their own
// alphas alpha_k = 1 - exp(-(l/K) act(v_k)) at their ray distances t_k,
//   d = sum_k prod_{j<k} (1 - alpha_j) alpha_k t_k
template <int KT, int ACT, int NB>
__device__ __forceinline__ float segment_xd(const LdsBatch<NB>& B, int j, double dx, double dy,
                                            double dz, double a, double lseg, int Krt,
                                            float& dloc) {
  const int K = KT > 0 ? KT : Krt;
  const double step = 1.0 / (double)K;
  const float lK = (float)lseg / (float)K;
  float x = 0.f, P = 1.f, d = 0.f;
#pragma unroll
  for (int k = 0; k < (KT > 0 ? KT : SVR_MAX_K); ++k) {
    if (KT == 0 && k >= K) break;
    const double t = fma(((double)k + 0.5) * step, lseg, a);
    float qx, qy, qz;
    local_coord(B, j, t, dx, dy, dz, qx, qy, qz);
    const float xk = lK * act_f<ACT>(trilerp(B, j, qx, qy, qz));
    const float ak = alpha_of(xk);
    d = __fmaf_rn(P * ak, (float)t, d);
    P *= 1.f - ak;
    x += xk;
  }
  dloc = d;
  return x;
}

// local depth d of staged entry j and dd/dV for its 8 corner raw densities:
// dd/dalpha_k = P_k (t_k - E_{k+1}), P_k the product of (1 - alpha) before k
// and E_{k+1} the samples after k composited from k + 1 on;
// dalpha_k/dv_k = (1 - alpha_k) (l/K) act'(v_k); dv_k/dV_m = w_m(q_k)
template <int KT, int ACT, int NB>
__device__ __forceinline__ float segment_depth_grad(const LdsBatch<NB>& B, int j, double dx,
                                                    double dy, double dz, double a, double lseg,
                                                    int Krt, float dd[8]) {
  constexpr int KM = KT > 0 ? KT : SVR_MAX_K;
  const int K = KT > 0 ? KT : Krt;
  const double step = 1.0 / (double)K;
  const float lK = (float)lseg / (float)K;
  float al[KM], tk[KM], Pk[KM], ck[KM];
  float P = 1.f, d = 0.f;
#pragma unroll
  for (int k = 0; k < KM; ++k) {
    al[k] = 0.f; tk[k] = 0.f; Pk[k] = 0.f; ck[k] = 0.f;
    if (KT == 0 && k >= K) continue;
    const double t = fma(((double)k + 0.5) * step, lseg, a);
    float qx, qy, qz;
    local_coord(B, j, t, dx, dy, dz, qx, qy, qz);
    const float v = trilerp(B, j, qx, qy, qz);
    al[k] = alpha_of(lK * act_f<ACT>(v));
    ck[k] = (1.f - al[k]) * lK * act_df<ACT>(v);  // dalpha_k / dv_k
    tk[k] = (float)t;
    Pk[k] = P;
    d = __fmaf_rn(P * al[k], tk[k], d);
    P *= 1.f - al[k];
  }
  float E = 0.f;
#pragma unroll
  for (int k = KM - 1; k >= 0; --k) {
    if (KT == 0 && k >= K) continue;
    ck[k] *= Pk[k] * (tk[k] - E);
    E = __fmaf_rn(al[k], tk[k] - E, E);
  }
#pragma unroll
  for (int m = 0; m < 8; ++m) dd[m] = 0.f;
#pragma unroll
  for (int k = 0; k < KM; ++k) {
    if (KT == 0 && k >= K) break;
    const double t = fma(((double)k + 0.5) * step, lseg, a);
    float qx, qy, qz;
    local_coord(B, j, t, dx, dy, dz, qx, qy, qz);
    const float c = ck[k];
    const float px = 1.f - qx, py = 1.f - qy, pz = 1.f - qz;
    const float a00 = c * px * py, a01 = c * px * qy, a10 = c * qx * py, a11 = c * qx * qy;
    dd[0] = __fmaf_rn(a00, pz, dd[0]); dd[1] = __fmaf_rn(a00, qz, dd[1]);
    dd[2] = __fmaf_rn(a01, pz, dd[2]); dd[3] = __fmaf_rn(a01, qz, dd[3]);
    dd[4] = __fmaf_rn(a10, pz, dd[4]); dd[5] = __fmaf_rn(a10, qz, dd[5]);
    dd[6] = __fmaf_rn(a11, pz, dd[6]); dd[7] = __fmaf_rn(a11, qz, dd[7]);
  }
  return d;
}

// ---------------------------------------------------------------------------
// Forward, dense form.  Hits are sparse in a wave (a voxel a few pixels wide
// covers a handful of the 64 pixels of a block), so the per-hit work is not
// run entry by entry with most lanes idle.  Per staged batch, each wave
//   A. walks the entries touching its block once: lanes whose pixel lies in
//      the voxel's projected rectangle (and whose sign pattern matches, and
//      which have not terminated) append the entry to their own list, and a
//      wave-wide task queue records (lane, list slot, entry) in entry order.
//      The entries' sign/block word and rectangle come from registers (one
//      LDS read per 64 entries, then v_readlane), so the walk has no LDS
//      round trip per entry;
//   B. takes the queued candidates 64 at a time, one per lane: the fp64
//      ray-box test with the owning pixel's ray and, for a hit, the optical
//      depth x over K samples (written back to the owner's list, -1 on a
//      miss);
//   C. lets every lane composite its own list in entry order (the only
//      sequential part: a few operations per hit), after loading the whole
//      list (optical depths, entries, colours) at once.
// A lane list holding kListCap candidates triggers B and C early, so order
// and early termination are those of the plain per-pixel walk.
template <int TS, bool AUX = false>
struct DenseCfg {
  // 32x32 tiles with depth and normal lists would exceed the LDS
  static constexpr int kListCap = (TS == 32 && AUX) ? 4 : 8;
};

// queue word: owner lane | list slot (3 bits) << kSlotShift | staged entry
// << kEntryShift; 16 bits when a batch holds at most 64 entries, else 32
template <int NB>
struct QueueWord {
  static constexpr bool kSmall = NB <= 64;
  using T = typename std::conditional<kSmall, uint16_t, uint32_t>::type;
  static constexpr int kSlotShift = kSmall ? 6 : 8;
  static constexpr int kEntryShift = kSmall ? 9 : 16;
};

template <int CAP, bool AUX, int NB>
struct alignas(16) WaveLists {
  static_assert(CAP == 4 || CAP == 8, "list slots are loaded 4 at a time");
  typename QueueWord<NB>::T queue[64 * CAP];  // task -> (owner lane, list slot, entry)
  float xl[64][CAP];         // per lane: optical depth of each candidate (< 0: a miss)
  float dl[AUX ? 64 : 1][AUX ? CAP : 1];  // its local depth (depth images only)
  uint8_t jl[64][CAP];       // per lane: staged entry index of each candidate
};

// value of v in lane src (all lanes of the wave must execute this)
__device__ __forceinline__ double lane_f64(double v, int src) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_ds_bpermute(src << 2, (int)(uint32_t)b);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_ds_bpermute(src << 2, (int)(uint32_t)(b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

__device__ __forceinline__ uint32_t lane_rank(unsigned long long mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// b in the lanes whose bit is set in the wave-uniform mask m, a elsewhere
// (one v_cndmask with m as its lane mask)
__device__ __forceinline__ int select_lanes(int a, int b, unsigned long long m) {
  int r;
  asm("v_cndmask_b32_e64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "s"(m));
  return r;
}

// 64-bit mask of the pixels of the 8x8 block at (bu0, bv0) (bit 8 y + x)
// that lie in the pixel rectangle rx = u0 | u1 << 16, ry = v0 | v1 << 16
__device__ __forceinline__ void block_rect_mask(uint32_t rx, uint32_t ry, int bu0, int bv0,
                                                uint32_t& mlo, uint32_t& mhi) {
  mlo = mhi = 0u;
  const int cu0 = max((int)(rx & 0xffffu) - bu0, 0), cu1 = min((int)(rx >> 16) - bu0, 7);
  const int cv0 = max((int)(ry & 0xffffu) - bv0, 0), cv1 = min((int)(ry >> 16) - bv0, 7);
  if (cu0 <= cu1 && cv0 <= cv1) {
    uint32_t row = ((2u << cu1) - 1u) & ~((1u << cu0) - 1u);
    row |= row << 8;
    row |= row << 16;
    const unsigned long long rows =
        (cv1 == 7 ? ~0ull : ((1ull << (8 * (cv1 + 1))) - 1ull)) & ~((1ull << (8 * cv0)) - 1ull);
    mlo = row & (uint32_t)rows;
    mhi = row & (uint32_t)(rows >> 32);
  }
}


// STATS: count, per frame, the (pixel, entry) pairs of matching sign pattern
// the method walks, the ray-box tests this kernel executes (candidates after
// the rectangle test), and the composited hits (into stats[0..2]); no outputs.
template <int TS, int KT, int ACT, bool STATS, bool AUX>
__device__ __forceinline__ void render_tile_fwd(const RenderArgs& A, int g,
                                                LdsBatch<TileGeom<TS>::kBatch>& B,
                                                uint32_t* mw,  // per staged entry: max blending weight (float bits)
                                                WaveLists<DenseCfg<TS, AUX>::kListCap, AUX, TileGeom<TS>::kBatch>* WLs) {
  using G = TileGeom<TS>;
  constexpr int NB = G::kBatch;
  constexpr int CAP = DenseCfg<TS, AUX>::kListCap;
  const int ci = find_cam_r(A.cams, g);
  const DevCam& c = A.cams.c[ci];
  const int tl = g - c.tile_off;
  const int tx = tl % c.ntx, ty = tl / c.ntx;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int qu0 = tx * TS, qv0 = ty * TS;
  const PixelRay r = make_ray<TS>(c, qu0, qv0, w, lane);
  using QW = QueueWord<NB>;
  WaveLists<CAP, AUX, NB>& WL = WLs[w];
  const int bu0 = qu0 + (w % G::kBpr) * 8, bv0 = qv0 + (w / G::kBpr) * 8;  // this wave's block

  const uint2 rg = A.range[g];
  const uint32_t start = rg.x, end = rg.y;
  float tau = 0.f, Tr = 1.f, C0 = 0.f, C1 = 0.f, C2 = 0.f;
  float D = 0.f, N0 = 0.f, N1 = 0.f, N2 = 0.f;  // depth and normal images
  uint32_t last = start;
  bool done = !r.inside;
  uint32_t n_pairs = 0, n_tests = 0, n_hits = 0;
  // heavy tile: record (tau, colour so far) at every chunk boundary passed
  const uint32_t sb = STATS ? kNoSplit : A.split_base[g];
  float4* const ck = A.ckpt + (int64_t)(sb == kNoSplit ? 0u : sb) * (TS * TS) + tid;
  float4* const ck_aux = A.ckpt_aux + (int64_t)(sb == kNoSplit ? 0u : sb) * (TS * TS) + tid;
  uint32_t n_ck = 0;

  for (uint32_t b0 = start; b0 < end; b0 += NB) {
    const uint32_t i = b0 + tid;
    if (tid < NB && i < end) {
      stage_entry<TS>(B, tid, A.vals[i], ci, A.n_cams, c, A.rec, A.rect, qu0, qv0);
      mw[tid] = 0u;
    }
    __syncthreads();
    const int n = (int)min((uint32_t)NB, end - b0);
    int cnt = 0;    // this lane's list length
    uint32_t nq = 0;  // queue length (wave-uniform)
    auto flush = [&]() {
      wave_sync_lds();
      // B: candidates, one per lane; the owner's ray comes from its lane
      // (ds_bpermute, with every lane of the wave taking part)
      for (uint32_t tb = 0; tb < nq; tb += 64) {
        const bool act = tb + lane < nq;
        const uint32_t q = act ? (uint32_t)WL.queue[tb + lane] : 0u;
        const int ow = (int)(q & 63u), k = (int)((q >> QW::kSlotShift) & 7u);
        const int j = (int)(q >> QW::kEntryShift);
        const double dx = lane_f64(r.dx, ow), dy = lane_f64(r.dy, ow), dz = lane_f64(r.dz, ow);
        const double idx = lane_f64(r.idx, ow), idy = lane_f64(r.idy, ow);
        const double idz = lane_f64(r.idz, ow);
        if (act) {
          double a, bb;
          float x = -1.f;
          if (slab(B, j, idx, idy, idz, a, bb)) {
            if (AUX) {
              float dloc;
              x = segment_xd<KT, ACT>(B, j, dx, dy, dz, a, bb - a, A.K, dloc);
              WL.dl[AUX ? ow : 0][AUX ? k : 0] = dloc;
            } else {
              x = segment_x<KT, ACT, false>(B, j, dx, dy, dz, a, bb - a, A.K, nullptr);
            }
          }
          WL.xl[ow][k] = x;
          if (STATS) ++n_tests;
        }
      }
      wave_sync_lds();
      // C: each lane composites its own list in entry order; the list is
      // loaded first (4 slots per LDS read) so the loop waits on LDS once
      float xs[CAP];
      uint32_t jw[CAP / 4];
#pragma unroll
      for (int h = 0; h < CAP / 4; ++h) {
        const float4 xv = reinterpret_cast<const float4*>(&WL.xl[lane][0])[h];
        xs[4 * h + 0] = xv.x; xs[4 * h + 1] = xv.y; xs[4 * h + 2] = xv.z; xs[4 * h + 3] = xv.w;
        jw[h] = reinterpret_cast<const uint32_t*>(&WL.jl[lane][0])[h];
      }
      float4 cc[CAP];
#pragma unroll
      for (int k = 0; k < CAP; ++k)
        cc[k] = B.col[(jw[k >> 2] >> (8 * (k & 3))) & (uint32_t)(NB - 1)];
#pragma unroll
      for (int k = 0; k < CAP; ++k) {
        if (__ballot(k < cnt) == 0ull) break;
        if (k < cnt && !done) {
          const float x = xs[k];
          if (x >= 0.f) {
            const int j = (int)((jw[k >> 2] >> (8 * (k & 3))) & (uint32_t)(NB - 1));
            const float wgt = Tr * alpha_of(x);
            if (A.max_weight) atomicMax(&mw[j], __float_as_uint(wgt));
            C0 = __fmaf_rn(wgt, cc[k].x, C0);
            C1 = __fmaf_rn(wgt, cc[k].y, C1);
            C2 = __fmaf_rn(wgt, cc[k].z, C2);
            if (AUX) {
              float nv[3];
              staged_normal(B, j, nv);
              D = __fmaf_rn(Tr, WL.dl[AUX ? lane : 0][AUX ? k : 0], D);
              N0 = __fmaf_rn(wgt, nv[0], N0);
              N1 = __fmaf_rn(wgt, nv[1], N1);
              N2 = __fmaf_rn(wgt, nv[2], N2);
            }
            tau += x;
            Tr = __expf(-tau);
            last = b0 + (uint32_t)j + 1u;
            if (STATS) ++n_hits;
            if (Tr < A.t_stop) done = true;
          }
        }
      }
      wave_sync_lds();
      cnt = 0;
      nq = 0;
    };
    // A: candidate lists.  64 entries at a time, entry jb + e held by lane e
    // with its sign/block word and the mask of this wave's pixels inside its
    // rectangle; per entry the candidates are that mask & the pixels of its
    // sign pattern & the pixels still compositing
    for (int jb = 0; jb < n; jb += 64) {
      const int jn = min(64, n - jb);
      uint32_t meta_v = 0u, mlo = 0u, mhi = 0u;
      if (lane < jn) {
        meta_v = B.meta[jb + lane];
        if ((meta_v >> (3 + w)) & 1u) block_rect_mask(B.rx[jb + lane], B.ry[jb + lane], bu0, bv0, mlo, mhi);
      }
      unsigned long long live = __ballot(!done);
      for (int jj = 0; jj < jn; ++jj) {
        const uint32_t meta = (uint32_t)__builtin_amdgcn_readlane((int)meta_v, jj);
        if (STATS && !done && (meta & 7u) == r.spat) ++n_pairs;
        const unsigned long long rm =
            ((unsigned long long)(uint32_t)__builtin_amdgcn_readlane((int)mhi, jj) << 32) |
            (uint32_t)__builtin_amdgcn_readlane((int)mlo, jj);
        if ((rm & live) == 0ull) continue;
        const unsigned long long m = rm & live & __ballot(r.spat == (meta & 7u));
        if (m == 0ull) continue;
        const bool cand = ((m >> lane) & 1ull) != 0ull;
        const int j = jb + jj;
        if (cand) {
          WL.queue[nq + lane_rank(m)] =
              (typename QW::T)((uint32_t)lane | ((uint32_t)cnt << QW::kSlotShift) |
                               ((uint32_t)j << QW::kEntryShift));
          WL.jl[lane][cnt] = (uint8_t)j;
          ++cnt;
        }
        nq += (uint32_t)__popcll(m);
        if (__ballot(cnt == CAP) != 0ull) {
          flush();
          live = __ballot(!done);
        }
      }
    }
    if (nq > 0) flush();
    if (sb != kNoSplit) {
      const uint32_t bend = b0 + NB;
      if (bend < end && ((bend - start) & (kBwdChunk - 1)) == 0) {
        ck[(int64_t)n_ck * (TS * TS)] = make_float4(tau, C0, C1, C2);
        if (AUX) ck_aux[(int64_t)n_ck * (TS * TS)] = make_float4(D, N0, N1, N2);
        ++n_ck;
      }
    }
    const bool all_done = __syncthreads_and(done);
    // the batch's maxima, one global atomic per entry with a composited hit
    if (!STATS && A.max_weight && tid < n && mw[tid] != 0u)
      atomicMax(A.max_weight + __float_as_uint(B.col[tid].w), mw[tid]);
    if (all_done) break;
  }
  // the backward wants the colour still to come: final minus so far
  for (uint32_t k = 0; k < n_ck; ++k) {
    const float4 q = ck[(int64_t)k * (TS * TS)];
    ck[(int64_t)k * (TS * TS)] = make_float4(q.x, C0 - q.y, C1 - q.z, C2 - q.w);
    if (AUX) {
      const float4 e = ck_aux[(int64_t)k * (TS * TS)];
      ck_aux[(int64_t)k * (TS * TS)] = make_float4(D - e.x, N0 - e.y, N1 - e.z, N2 - e.w);
    }
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
      atomicAdd(A.stats + 0, a0);
      atomicAdd(A.stats + 1, a1);
      atomicAdd(A.stats + 2, a2);
    }
    return;
  }
  if (r.inside) {
    const int64_t p = c.pix_off + (int64_t)r.v * c.W + r.u;
    A.rgba[p] = make_float4(C0, C1, C2, 1.f - Tr);
    A.px_tau[p] = tau;
    A.px_last[p] = last;
    if (AUX && A.depth) A.depth[p] = D;
    if (AUX && A.normal) {
      A.normal[3 * p + 0] = N0;
      A.normal[3 * p + 1] = N1;
      A.normal[3 * p + 2] = N2;
    }
  }
}

template <int TS, int KT, int ACT, bool STATS, bool AUX>
__global__ __launch_bounds__(TS * TS) void k_render_fwd(RenderArgs A) {
  __shared__ LdsBatch<TileGeom<TS>::kBatch> B;
  __shared__ uint32_t mw[TileGeom<TS>::kBatch];
  __shared__ WaveLists<DenseCfg<TS, AUX>::kListCap, AUX, TileGeom<TS>::kBatch> WL[TileGeom<TS>::kWaves];
  __shared__ int s_tile;
  if (!A.persistent) {
    if ((int)blockIdx.x < A.T) render_tile_fwd<TS, KT, ACT, STATS, AUX>(A, A.order[blockIdx.x], B, mw, WL);
    return;
  }
  while (true) {
    if (threadIdx.x == 0) s_tile = next_tile(A.work, A.T);
    __syncthreads();
    const int p = s_tile;
    if (p < 0) break;
    const int g = A.order[p];
    render_tile_fwd<TS, KT, ACT, STATS, AUX>(A, g, B, mw, WL);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Wave sum of 16 per-lane values by recursive halving with gfx950 cross-lane
// VALU operations (no LDS): at each step a lane keeps one half of its values
// and adds its partner lane's copy of that half.
//   step 1: v_permlane32_swap pairs lane L with L ^ 32  (8 pairs -> 8 values)
//   step 2: v_permlane16_swap pairs 16-lane rows 0<->1, 2<->3 (-> 4 values)
//   step 3: DPP row_mirror pairs i <-> 15 - i in a row     (-> 2 values)
//   step 4: DPP row_half_mirror pairs i <-> 7 - i          (-> 1 value)
//   step 5: two quad DPP adds (xor 1, xor 2) finish the sum.
// Lane L then holds the wave total of value (L >> 2) & 15; lanes 4 i hold
// value i.  About 35 VALU instructions in all.
__device__ __forceinline__ float swap32_sum(float lo, float hi) {
  // upper 32 lanes of the first operand <-> lower 32 lanes of the second
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(lo), __float_as_uint(hi), false,
                                                  false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

__device__ __forceinline__ float swap16_sum(float lo, float hi) {
  // odd rows of the first operand <-> even rows of the second
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(lo), __float_as_uint(hi), false,
                                                  false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

template <int CTRL>
__device__ __forceinline__ float dpp(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xf, 0xf, false));
}

template <int CTRL>
__device__ __forceinline__ float dpp_pair_sum(float lo, float hi, bool upper) {
  const float keep = upper ? hi : lo;
  const float send = upper ? lo : hi;
  return keep + dpp<CTRL>(send);
}

constexpr int kDppRowMirror = 0x140;
constexpr int kDppRowShr1 = 0x111;
constexpr int kDppRowShr2 = 0x112;
constexpr int kDppRowShr4 = 0x114;
constexpr int kDppRowShr8 = 0x118;
constexpr int kDppWaveShr1 = 0x138;   // whole wave, lane L takes lane L - 1
constexpr int kDppRowBcast15 = 0x142;  // lane 15 of a row to the next row
constexpr int kDppRowBcast31 = 0x143;  // lane 31 to rows 2 and 3
constexpr int kDppRowHalfMirror = 0x141;
constexpr int kDppQuadXor1 = 0xB1;  // quad_perm [1,0,3,2]
constexpr int kDppQuadXor2 = 0x4E;  // quad_perm [2,3,0,1]

// DPP move of a 32-bit value; lanes with no source (and rows outside
// ROW_MASK) read 0
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ uint32_t dpp_u(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, ROW_MASK, 0xf, true);
}

__device__ __forceinline__ float wave_reduce16(const float (&g)[16]) {
  const int lane = threadIdx.x & 63;
  const float s0 = swap32_sum(g[0], g[8]), s1 = swap32_sum(g[1], g[9]);
  const float s2 = swap32_sum(g[2], g[10]), s3 = swap32_sum(g[3], g[11]);
  const float s4 = swap32_sum(g[4], g[12]), s5 = swap32_sum(g[5], g[13]);
  const float s6 = swap32_sum(g[6], g[14]), s7 = swap32_sum(g[7], g[15]);
  const float t0 = swap16_sum(s0, s4), t1 = swap16_sum(s1, s5);
  const float t2 = swap16_sum(s2, s6), t3 = swap16_sum(s3, s7);
  const bool u8 = (lane & 8) != 0, u4 = (lane & 4) != 0;
  const float w0 = dpp_pair_sum<kDppRowMirror>(t0, t2, u8);
  const float w1 = dpp_pair_sum<kDppRowMirror>(t1, t3, u8);
  float x = dpp_pair_sum<kDppRowHalfMirror>(w0, w1, u4);
  x += dpp<kDppQuadXor1>(x);
  x += dpp<kDppQuadXor2>(x);
  return x;
}

// The same for 12 values (no depth/normal gradients): 6 permlane32 swaps,
// 3 permlane16 swaps, then the row mirrors on 3 values (one slot padded with
// zero) and the quad adds; about 29 VALU instructions.  Lane L ends up with
// value red12_slot(L) (see there); lanes with (L >> 2) & 3 == 3 hold nothing.
__device__ __forceinline__ float wave_reduce12(const float (&g)[16]) {
  const int lane = threadIdx.x & 63;
  const float s0 = swap32_sum(g[0], g[6]), s1 = swap32_sum(g[1], g[7]);
  const float s2 = swap32_sum(g[2], g[8]), s3 = swap32_sum(g[3], g[9]);
  const float s4 = swap32_sum(g[4], g[10]), s5 = swap32_sum(g[5], g[11]);
  const float t0 = swap16_sum(s0, s3), t1 = swap16_sum(s1, s4), t2 = swap16_sum(s2, s5);
  const bool u8 = (lane & 8) != 0, u4 = (lane & 4) != 0;
  const float w0 = dpp_pair_sum<kDppRowMirror>(t0, t2, u8);
  const float w1 = dpp_pair_sum<kDppRowMirror>(t1, 0.f, u8);
  float x = dpp_pair_sum<kDppRowHalfMirror>(w0, w1, u4);
  x += dpp<kDppQuadXor1>(x);
  x += dpp<kDppQuadXor2>(x);
  return x;
}

// value index lane L holds after wave_reduce12: 6 (L >> 5) + 3 ((L >> 4) & 1)
// + i, i = 0, 1, 2 for (L >> 2) & 3 = 0, 1, 2 (and 3: none, returned as 15)
__device__ __forceinline__ int red12_slot(int lane) {
  const int q = (lane >> 2) & 3;
  return q == 3 ? 15 : 6 * (lane >> 5) + 3 * ((lane >> 4) & 1) + q;
}

// Backward of chunks [m_lo, m_hi) of tile g (entries [start + m_lo C,
// min(start + m_hi C, end)), C = kBwdChunk).  A pixel whose last composited
// entry lies beyond the range starts from the forward's checkpoint at the
// range's end (optical depth so far, colour still to come); the others start
// from their final state.
template <int TS, int KT, int ACT, bool AUX>
__device__ __forceinline__ void render_tile_bwd(const RenderArgs& A, int g, uint32_t m_lo,
                                                uint32_t m_hi,
                                                LdsBatch<TileGeom<TS>::kBatch>& B,
                                                uint32_t& s_lmax) {
  using G = TileGeom<TS>;
  constexpr int NB = G::kBatch;
  const int ci = find_cam_r(A.cams, g);
  const DevCam& c = A.cams.c[ci];
  const int tl = g - c.tile_off;
  const int tx = tl % c.ntx, ty = tl / c.ntx;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int qu0 = tx * TS, qv0 = ty * TS;
  const PixelRay r = make_ray<TS>(c, qu0, qv0, w, lane);
  // reduced value this lane ends up holding: 12 values without depth and
  // normal images, 16 with them
  const int slot = AUX ? (lane >> 2) & 15 : red12_slot(lane);
  const bool prio = A.priority != nullptr;
  // values: 0-7 corners, 8-10 colour, 11 priority, 12-14 dL/dn (depth and normal)
  const bool writer = (lane & 3) == 0 &&
                      (slot < 11 || (slot == 11 && prio) || (AUX && slot >= 12 && slot < 15));
  auto reduce = [&](const float (&g)[16]) { return AUX ? wave_reduce16(g) : wave_reduce12(g); };

  const uint2 rg = A.range[g];
  const uint32_t e_lo = rg.x + m_lo * (uint32_t)kBwdChunk;
  const uint32_t e_hi = min(rg.x + m_hi * (uint32_t)kBwdChunk, rg.y);
  float tau = 0.f, gr = 0.f, gg = 0.f, gb = 0.f, ga = 0.f, Tfin = 1.f, tau_end = 0.f;
  float U0 = 0.f, U1 = 0.f, U2 = 0.f;  // colour composited after the current entry
  float UD = 0.f, UN0 = 0.f, UN1 = 0.f, UN2 = 0.f;  // the same for depth and normal
  float gD = 0.f, gN0 = 0.f, gN1 = 0.f, gN2 = 0.f;
  uint32_t last = e_lo;
  if (r.inside) {
    const int64_t p = c.pix_off + (int64_t)r.v * c.W + r.u;
    const float tau_fin = A.px_tau[p];
    tau_end = tau_fin;
    const uint32_t lp = A.px_last[p];
    const float4 gq = A.grad_rgba[p];
    gr = gq.x; gg = gq.y; gb = gq.z; ga = gq.w;
    if (AUX) {
      if (A.grad_depth) gD = A.grad_depth[p];
      if (A.grad_normal) {
        gN0 = A.grad_normal[3 * p + 0];
        gN1 = A.grad_normal[3 * p + 1];
        gN2 = A.grad_normal[3 * p + 2];
      }
    }
    Tfin = __expf(-tau_fin);
    if (lp > e_hi) {  // only in a split chunk (e_hi < end), whose tile has checkpoints
      const int64_t slot_px = ((int64_t)A.split_base[g] + m_hi - 1) * (TS * TS) + tid;
      const float4 q = A.ckpt[slot_px];
      tau = q.x; U0 = q.y; U1 = q.z; U2 = q.w;
      if (AUX) {
        const float4 e = A.ckpt_aux[slot_px];
        UD = e.x; UN0 = e.y; UN1 = e.z; UN2 = e.w;
      }
      last = e_hi;
    } else {
      tau = tau_fin;
      last = lp;
    }
  }
  // transmittance just behind the current hit: exp(-tau) before tau drops by
  // the hit's x, carried from one hit to the one before it
  float Tnext = __expf(-tau);
  if (tid == 0) s_lmax = e_lo;
  __syncthreads();
  if (last > e_lo) atomicMax(&s_lmax, last);
  __syncthreads();
  const uint32_t lmax = s_lmax;

  uint32_t bend = lmax;
  while (bend > e_lo) {
    const uint32_t b0 = bend - min((uint32_t)NB, bend - e_lo);
    const int n = (int)(bend - b0);
    bend = b0;
    if (tid < n)
      stage_entry<TS>(B, tid, A.vals[b0 + tid], ci, A.n_cams, c, A.rec, A.rect, qu0, qv0);
    __syncthreads();
    // one hit: step the pixel's reverse state over staged entry j (hit on
    // [a, bb]) and write its gradients into gv[0..14]
    auto hit_grads = [&](int j, double a, double bb, float (&gv)[16]) {
      constexpr bool kTwoPhase = KT > 0 && !AUX;
      constexpr int KQ = KT > 0 ? KT : 1;
      float dw[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      float qs[KQ][3], dks[KQ];
      const double lseg = bb - a;
      const float x = kTwoPhase
                          ? segment_samples<KQ, ACT>(B, j, r.dx, r.dy, r.dz, a, lseg, qs, dks)
                          : segment_x<KT, ACT, true>(B, j, r.dx, r.dy, r.dz, a, lseg, A.K, dw);
      const float lK = (float)lseg / (float)(KT > 0 ? KT : A.K);
      const float alpha = alpha_of(x);
      tau -= x;
      const float Ti = __expf(-tau);
      const float4 cj = B.col[j];
      const float cr = cj.x, cg = cj.y, cb = cj.z;
      const float wgt = Ti * alpha;
      gv[8] = gr * wgt; gv[9] = gg * wgt; gv[10] = gb * wgt;
      float dLdx = gr * (Tnext * cr - U0) + gg * (Tnext * cg - U1) +
                   gb * (Tnext * cb - U2) + ga * Tfin;
      float dd[8], dloc = 0.f, nv[3] = {0.f, 0.f, 0.f};
      if (AUX) {
        // depth: D = sum T_i d_i (d_i through its sample alphas; the hits
        // behind through T); normal: N = sum T_i alpha_i n_i, as the colour
        dloc = segment_depth_grad<KT, ACT>(B, j, r.dx, r.dy, r.dz, a, lseg, A.K, dd);
        staged_normal(B, j, nv);
        dLdx += -gD * UD + gN0 * (Tnext * nv[0] - UN0) + gN1 * (Tnext * nv[1] - UN1) +
                gN2 * (Tnext * nv[2] - UN2);
        gv[12] = wgt * gN0;
        gv[13] = wgt * gN1;
        gv[14] = wgt * gN2;
      }
      if (prio) {
        // |alpha dL/dalpha| (eq. priority) = |T_i alpha <g, c - S> + g_A (e^{-(tau_fin - x)}
        // - T_fin)|, S = U / T_{i+1} the colour behind seen from just behind (0 when
        // T_{i+1} underflows: then nothing is composited behind and U = 0)
        const float iT = Tnext > 0.f ? 1.f / Tnext : 0.f;
        gv[11] = fabsf(wgt * (gr * (cr - U0 * iT) + gg * (cg - U1 * iT) + gb * (cb - U2 * iT)) +
                       ga * (__expf(x - tau_end) - Tfin));
      }
      U0 = __fmaf_rn(wgt, cr, U0);
      U1 = __fmaf_rn(wgt, cg, U1);
      U2 = __fmaf_rn(wgt, cb, U2);
      if (AUX) {
        UD = __fmaf_rn(Ti, dloc, UD);
        UN0 = __fmaf_rn(wgt, nv[0], UN0);
        UN1 = __fmaf_rn(wgt, nv[1], UN1);
        UN2 = __fmaf_rn(wgt, nv[2], UN2);
      }
      Tnext = Ti;
      const float f = dLdx * lK;
      if (kTwoPhase) {
        corner_grads<KQ>(qs, dks, f, gv);
      } else {
#pragma unroll
        for (int m = 0; m < 8; ++m) gv[m] = f * dw[m];
      }
      if (AUX) {
        const float gt = gD * Ti;
#pragma unroll
        for (int m = 0; m < 8; ++m) gv[m] = __fmaf_rn(gt, dd[m], gv[m]);
      }
    };
    // the wave total of reduced value `slot` of voxel vid goes to its gradient
    auto flush_grads = [&](float tot, uint32_t vid) {
      if (writer) {
        float* dst = slot < 8    ? A.g_corner + (int64_t)vid * 8 + slot
                     : slot < 11 ? A.g_rgb + ((int64_t)vid * A.n_cams + ci) * 3 + (slot - 8)
                     : slot < 12 ? A.priority + vid
                                 : A.g_nrm + (int64_t)vid * 3 + (slot - 12);
        unsafeAtomicAdd(dst, tot);
      }
    };
    if (!kGroupedBwd) {
      // 64 entries' voxel ids at a time in registers (a scalar base address
      // for the gradient atomics)
      uint32_t vid_v = 0u;
      for (int j = n - 1; j >= 0; --j) {
        if (j == n - 1 || (j & 63) == 63) {
          const int jb = j & ~63;
          vid_v = jb + lane < n ? __float_as_uint(B.col[jb + lane].w) : 0u;
        }
        const uint32_t meta = __builtin_amdgcn_readfirstlane(B.meta[j]);
        if (!((meta >> (3 + w)) & 1u)) continue;
        double a = 0.0, bb = 0.0;
        bool hit = (b0 + (uint32_t)j < last) && ((meta & 7u) == r.spat);
        if (hit) hit = slab(B, j, r.idx, r.idy, r.idz, a, bb);
        if (__ballot(hit) == 0ull) continue;
        float gv[16];
#pragma unroll
        for (int m = 0; m < 16; ++m) gv[m] = 0.f;
        if (hit) hit_grads(j, a, bb, gv);
        flush_grads(reduce(gv), (uint32_t)__builtin_amdgcn_readlane((int)vid_v, j & 63));
      }
    } else {
      // Grouped walk: 64 entries at a time, entry e of the chunk held by
      // lane e (entry top - e, so lane order is the reverse walk order) with
      // the mask of the block's pixels inside its projected rectangle.  An
      // entry whose mask is disjoint from the masks of every entry still
      // pending before it is the next entry of each of its pixels, so all
      // such entries are walked together, one per pixel lane: the hit path
      // runs once per group instead of once per entry (groups hold about
      // two entries on the benchmark scenes), and each entry's gradients are
      // then summed over its own lanes.
      const int bu0 = qu0 + (w % G::kBpr) * 8, bv0 = qv0 + (w / G::kBpr) * 8;
      for (int top = n - 1; top >= 0; top -= 64) {
        const int j_e = top - lane;  // this lane's entry (as an entry lane)
        uint32_t mlo = 0u, mhi = 0u, vid_e = 0u;
        if (j_e >= 0) {
          if ((B.meta[j_e] >> (3 + w)) & 1u) block_rect_mask(B.rx[j_e], B.ry[j_e], bu0, bv0, mlo, mhi);
          vid_e = __float_as_uint(B.col[j_e].w);
        }
        while (__ballot((mlo | mhi) != 0u) != 0ull) {
          // inclusive prefix OR of the masks in lane order, then exclusive
          uint32_t ilo = mlo, ihi = mhi;
          ilo |= dpp_u<kDppRowShr1>(ilo); ihi |= dpp_u<kDppRowShr1>(ihi);
          ilo |= dpp_u<kDppRowShr2>(ilo); ihi |= dpp_u<kDppRowShr2>(ihi);
          ilo |= dpp_u<kDppRowShr4>(ilo); ihi |= dpp_u<kDppRowShr4>(ihi);
          ilo |= dpp_u<kDppRowShr8>(ilo); ihi |= dpp_u<kDppRowShr8>(ihi);
          ilo |= dpp_u<kDppRowBcast15, 0xa>(ilo); ihi |= dpp_u<kDppRowBcast15, 0xa>(ihi);
          ilo |= dpp_u<kDppRowBcast31, 0xc>(ilo); ihi |= dpp_u<kDppRowBcast31, 0xc>(ihi);
          const uint32_t elo = dpp_u<kDppWaveShr1>(ilo), ehi = dpp_u<kDppWaveShr1>(ihi);
          const bool elig = (mlo | mhi) != 0u && ((mlo & elo) | (mhi & ehi)) == 0u;
          const unsigned long long E = __ballot(elig);
          // the group entry (lane) that holds this pixel, -1 if none
          int my = -1;
          for (unsigned long long es = E; es != 0ull; es &= es - 1ull) {
            const int e = __builtin_ctzll(es);
            const unsigned long long me =
                ((unsigned long long)(uint32_t)__builtin_amdgcn_readlane((int)mhi, e) << 32) |
                (uint32_t)__builtin_amdgcn_readlane((int)mlo, e);
            my = select_lanes(my, e, me);
          }
          if (elig) { mlo = 0u; mhi = 0u; }
          const int j = top - my;
          double a = 0.0, bb = 0.0;
          bool hit = false;
          if (my >= 0) {
            hit = (b0 + (uint32_t)j < last) && ((B.meta[j] & 7u) == r.spat);
            if (hit) hit = slab(B, j, r.idx, r.idy, r.idz, a, bb);
          }
          if (__ballot(hit) == 0ull) continue;
          float gv[16];
#pragma unroll
          for (int m = 0; m < 16; ++m) gv[m] = 0.f;
          if (hit) hit_grads(j, a, bb, gv);
          if ((E & (E - 1ull)) == 0ull) {
            // one entry: the lanes that did not hit it hold zeros already
            flush_grads(reduce(gv), (uint32_t)__builtin_amdgcn_readlane((int)vid_e, __builtin_ctzll(E)));
            continue;
          }
          for (unsigned long long es = E; es != 0ull; es &= es - 1ull) {
            const int e = __builtin_ctzll(es);
            const bool mine = hit && my == e;
            if (__ballot(mine) == 0ull) continue;
            float ge[16];
#pragma unroll
            for (int m = 0; m < 16; ++m) ge[m] = mine ? gv[m] : 0.f;
            flush_grads(reduce(ge), (uint32_t)__builtin_amdgcn_readlane((int)vid_e, e));
          }
        }
      }
    }
    __syncthreads();
  }
}

// chunk item k: (tile, chunk), checked against the tile before use
template <int TS, int KT, int ACT, bool AUX>
__device__ __forceinline__ void bwd_split_item(const RenderArgs& A, uint32_t k,
                                               LdsBatch<TileGeom<TS>::kBatch>& B,
                                               uint32_t& s_lmax) {
  const uint2 it = A.split_items[k];
  if (it.x >= (uint32_t)A.T || A.split_base[it.x] == kNoSplit) return;
  const uint2 rg = A.range[it.x];
  const uint32_t nch = (rg.y - rg.x + kBwdChunk - 1) / kBwdChunk;
  if (it.y + 1 >= nch) return;
  render_tile_bwd<TS, KT, ACT, AUX>(A, (int)it.x, it.y, it.y + 1, B, s_lmax);
}

// a tile's whole range, or its last chunk when the others are chunk items
template <int TS, int KT, int ACT, bool AUX>
__device__ __forceinline__ void bwd_tile_rest(const RenderArgs& A, int g,
                                              LdsBatch<TileGeom<TS>::kBatch>& B,
                                              uint32_t& s_lmax) {
  const uint2 rg = A.range[g];
  const uint32_t nch = (rg.y - rg.x + kBwdChunk - 1) / kBwdChunk;
  const uint32_t m_lo = (A.split_base[g] == kNoSplit || nch == 0) ? 0u : nch - 1;
  render_tile_bwd<TS, KT, ACT, AUX>(A, g, m_lo, nch, B, s_lmax);
}

// 6 waves per SIMD for the 8x8 backward where its registers fit 80 without
// spilling (K = 1, or K = 2 with explin, no depth or normal images); its
// LDS (5.9 KB per wave) allows 6 as well
template <int TS, int KT, int ACT, bool AUX>
constexpr int bwd_min_waves() {
  return (TS == 8 && !AUX && (KT == 1 || (KT == 2 && ACT == SVR_ACT_EXPLIN))) ? 6 : 1;
}

template <int TS, int KT, int ACT, bool AUX>
__global__ __launch_bounds__(TS * TS, (bwd_min_waves<TS, KT, ACT, AUX>())) void k_render_bwd(RenderArgs A) {
  __shared__ LdsBatch<TileGeom<TS>::kBatch> B;
  __shared__ uint32_t s_lmax;
  __shared__ int s_tile;
  const uint32_t ns = min(*A.split_count, (uint32_t)A.max_split);
  if (!A.persistent) {
    // the first split_wgs workgroups take the chunk items, the others one
    // tile each (its last chunk if it is split) in render order
    const int b = (int)blockIdx.x;
    if (b < A.split_wgs) {
      for (uint32_t k = (uint32_t)b; k < ns; k += (uint32_t)A.split_wgs) {
        bwd_split_item<TS, KT, ACT, AUX>(A, k, B, s_lmax);
        __syncthreads();
      }
    } else if (b - A.split_wgs < A.T) {
      bwd_tile_rest<TS, KT, ACT, AUX>(A, (int)A.order[b - A.split_wgs], B, s_lmax);
    }
    return;
  }
  while (true) {  // chunk items first, then the tiles
    if (threadIdx.x == 0) s_tile = next_tile(A.work, (int)ns);
    __syncthreads();
    const int k = s_tile;
    if (k < 0) break;
    bwd_split_item<TS, KT, ACT, AUX>(A, (uint32_t)k, B, s_lmax);
    __syncthreads();
  }
  __syncthreads();  // every thread has read the last s_tile before it is reused
  while (true) {
    if (threadIdx.x == 0) s_tile = next_tile(A.work + 1, A.T);
    __syncthreads();
    const int p = s_tile;
    if (p < 0) break;
    bwd_tile_rest<TS, KT, ACT, AUX>(A, (int)A.order[p], B, s_lmax);
    __syncthreads();
  }
}

// SH and grid adjoint, one thread per voxel.  The (D+1)^2 x 3 SH gradients of
// the workgroup's 256 voxels are staged in LDS and written out as one
// contiguous, coalesced block: degree 3 in 16-byte pieces (rows of 13
// float4, so that the 16-byte accesses of 8 consecutive lanes fall in
// different banks), lower degrees float by float (odd row stride).
template <int D>
__global__ __launch_bounds__(kBlock) void k_sh_bwd(
    int64_t N, int n_cams, CamSet cams, const float* __restrict__ center,
    const int32_t* __restrict__ vox_grid, const uint32_t* __restrict__ count,
    const VoxRec* __restrict__ rec, const float* __restrict__ g_rgb,
    float* __restrict__ g_corner, float* __restrict__ grad_grid, float* __restrict__ grad_sh,
    const float* __restrict__ grid_raw, const float* __restrict__ g_nrm, int accumulate,
    int scatter, int vec_ok) {
  constexpr int NB = (D + 1) * (D + 1);
  constexpr int F = 3 * NB;
  constexpr bool kVec = F % 4 == 0;  // degree 3: 48 floats, 12 float4 (16-byte aligned output)
  constexpr int FP = kVec ? F + 4 : (F | 1);
  __shared__ __align__(16) float stage[kBlock * FP];
  const int64_t base = (int64_t)blockIdx.x * kBlock;
  const int64_t vid = base + threadIdx.x;
  if (grad_sh) {
    float acc[NB][3];
#pragma unroll
    for (int j = 0; j < NB; ++j) acc[j][0] = acc[j][1] = acc[j][2] = 0.f;
    if (vid < N) {
      const float cx = center[vid], cy = center[N + vid], cz = center[2 * N + vid];
      for (int ci = 0; ci < n_cams; ++ci) {
        const int64_t vv = vid * n_cams + ci;
        // the record and colour gradient are read with the count (both are
        // only used when it is non-zero)
        const uint32_t cnt = count[vv];
        const uint32_t bits = __float_as_uint(rec[vv].q3.w);
        const float gr0 = g_rgb[vv * 3 + 0], gr1 = g_rgb[vv * 3 + 1], gr2 = g_rgb[vv * 3 + 2];
        if (cnt == 0) continue;
        const DevCam& c = cams.c[ci];
        const float g3[3] = {(bits & 1u) ? gr0 : 0.f, (bits & 2u) ? gr1 : 0.f, (bits & 4u) ? gr2 : 0.f};
        const float rx = cx - c.o[0], ry = cy - c.o[1], rz = cz - c.o[2];
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
    }
    const int nv = (int)min((int64_t)kBlock, N - base);
    float* o = grad_sh + base * F;
    if (kVec && vec_ok) {
      float4* st4 = reinterpret_cast<float4*>(stage + threadIdx.x * FP);
#pragma unroll
      for (int q = 0; q < F / 4; ++q)
        st4[q] = make_float4(acc[(4 * q + 0) / 3][(4 * q + 0) % 3], acc[(4 * q + 1) / 3][(4 * q + 1) % 3],
                             acc[(4 * q + 2) / 3][(4 * q + 2) % 3], acc[(4 * q + 3) / 3][(4 * q + 3) % 3]);
      __syncthreads();
      constexpr int F4 = F / 4, FP4 = FP / 4;
      const float4* s4 = reinterpret_cast<const float4*>(stage);
      float4* o4 = reinterpret_cast<float4*>(o);
      for (int i = threadIdx.x; i < nv * F4; i += kBlock) {
        float4 v = s4[(i / F4) * FP4 + (i % F4)];
        if (accumulate) {
          const float4 p = o4[i];
          v.x += p.x; v.y += p.y; v.z += p.z; v.w += p.w;
        }
        o4[i] = v;
      }
    } else {
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        stage[threadIdx.x * FP + 3 * j + 0] = acc[j][0];
        stage[threadIdx.x * FP + 3 * j + 1] = acc[j][1];
        stage[threadIdx.x * FP + 3 * j + 2] = acc[j][2];
      }
      __syncthreads();
      if (accumulate) {
        for (int i = threadIdx.x; i < nv * F; i += kBlock) o[i] += stage[(i / F) * FP + (i % F)];
      } else {
        for (int i = threadIdx.x; i < nv * F; i += kBlock) o[i] = stage[(i / F) * FP + (i % F)];
      }
    }
  }
  if (g_nrm && vid < N) {
    // normal images: dL/dn of the voxel to its corners, n = g / |g| with g the
    // centre gradient; dL/dg = (dL/dn - n (n . dL/dn)) / |g| and
    // dg/dV_ijk = 0.25 (2i - 1, 2j - 1, 2k - 1) (Supp. details of voxel normal)
    const float gn0 = g_nrm[vid * 3 + 0], gn1 = g_nrm[vid * 3 + 1], gn2 = g_nrm[vid * 3 + 2];
    if (gn0 != 0.f || gn1 != 0.f || gn2 != 0.f) {
      float V[8], gc3[3];
#pragma unroll
      for (int m = 0; m < 8; ++m) V[m] = grid_raw[vox_grid[vid * 8 + m]];
      centre_gradient(V, gc3);
      const float g2 = gc3[0] * gc3[0] + gc3[1] * gc3[1] + gc3[2] * gc3[2];
      if (g2 > 0.f) {
        const float il = rsqrtf(g2);
        const float n0 = gc3[0] * il, n1 = gc3[1] * il, n2 = gc3[2] * il;
        const float nd = n0 * gn0 + n1 * gn1 + n2 * gn2;
        const float q0 = 0.25f * (gn0 - n0 * nd) * il, q1 = 0.25f * (gn1 - n1 * nd) * il,
                    q2 = 0.25f * (gn2 - n2 * nd) * il;
#pragma unroll
        for (int m = 0; m < 8; ++m)
          g_corner[vid * 8 + m] += (((m >> 2) & 1) ? q0 : -q0) + (((m >> 1) & 1) ? q1 : -q1) +
                                   ((m & 1) ? q2 : -q2);
      }
    }
  }
  if (grad_grid && scatter && vid < N) {
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
enum class RKind { kFwd, kStats, kBwd };

static RenderArgs render_args(const CamSet& cams, const svr_opts& o, const Layout& L, void* ws,
                              const uint32_t* vals) {
  RenderArgs A;
  A.cams = cams;
  A.T = L.T;
  A.n_cams = L.n_cams;
  A.K = o.K;
  A.persistent = L.persistent > 0 ? 1 : 0;
  A.t_stop = o.t_stop;
  A.range = at<uint2>(ws, L.tile_range);
  A.vals = vals;
  A.rec = at<VoxRec>(ws, L.rec);
  A.rect = at<uint2>(ws, L.rect);
  A.rgba = nullptr;
  A.px_tau = at<float>(ws, L.px_tau);
  A.px_last = at<uint32_t>(ws, L.px_last);
  A.stats = at<WsHeader>(ws, L.hdr)->stats;
  A.grad_rgba = nullptr;
  A.g_corner = at<float>(ws, L.g_corner);
  A.g_rgb = at<float>(ws, L.g_rgb);
  A.work = at<WsHeader>(ws, L.hdr)->work;
  A.order = at<uint32_t>(ws, L.tile_order);
  A.split_base = at<uint32_t>(ws, L.split_base);
  A.split_items = at<uint2>(ws, L.split_items);
  A.split_count = at<uint32_t>(ws, L.tile_range) + 2 * (int64_t)L.T + kOrderBuckets;
  A.ckpt = at<float4>(ws, L.ckpt);
  A.max_split = (int)L.max_split;
  A.split_wgs = (int)min((int64_t)kSplitWgs, L.max_split);
  A.max_weight = nullptr;
  A.priority = nullptr;
  A.depth = A.normal = nullptr;
  A.grad_depth = A.grad_normal = nullptr;
  A.ckpt_aux = at<float4>(ws, L.ckpt_aux);
  A.g_nrm = at<float>(ws, L.g_nrm);
  A.aux = 0;
  return A;
}

template <int TS, int KT, int ACT, bool AUX>
static void launch_kind(RKind kind, const RenderArgs& A, unsigned grid, hipStream_t s) {
  const dim3 blk(TS * TS);
  switch (kind) {
    case RKind::kFwd:
      SVR_LAUNCH("render_fwd", (k_render_fwd<TS, KT, ACT, false, AUX>), dim3(grid), blk, 0, s, A);
      break;
    case RKind::kStats:
      SVR_LAUNCH("render_stats", (k_render_fwd<TS, KT, ACT, true, false>), dim3(grid), blk, 0, s,
                 A);
      break;
    case RKind::kBwd:
      SVR_LAUNCH("render_bwd", (k_render_bwd<TS, KT, ACT, AUX>), dim3(grid), blk, 0, s, A);
      break;
  }
}

template <int TS, int KT, int ACT>
static void launch_kind(RKind kind, const RenderArgs& A, unsigned grid, hipStream_t s) {
  launch_kind<TS, KT, ACT, false>(kind, A, grid, s);
}

template <int TS, int ACT>
static void launch_k(RKind kind, const RenderArgs& A, unsigned grid, hipStream_t s) {
  // depth and normal images: kernels of their own (K = 1, 2, 3 compiled in,
  // other K at run time)
  if (A.aux && kind != RKind::kStats) {
    switch (A.K) {
      case 1: launch_kind<TS, 1, ACT, true>(kind, A, grid, s); break;
      case 2: launch_kind<TS, 2, ACT, true>(kind, A, grid, s); break;
      case 3: launch_kind<TS, 3, ACT, true>(kind, A, grid, s); break;
      default: launch_kind<TS, 0, ACT, true>(kind, A, grid, s); break;
    }
    return;
  }
  switch (A.K) {
    case 1: launch_kind<TS, 1, ACT>(kind, A, grid, s); break;
    case 2: launch_kind<TS, 2, ACT>(kind, A, grid, s); break;
    case 3: launch_kind<TS, 3, ACT>(kind, A, grid, s); break;
    default: launch_kind<TS, 0, ACT>(kind, A, grid, s); break;
  }
}

template <int TS>
static void launch_act(RKind kind, const RenderArgs& A, int act, unsigned grid, hipStream_t s) {
  if (act == SVR_ACT_SOFTPLUS) launch_k<TS, SVR_ACT_SOFTPLUS>(kind, A, grid, s);
  else launch_k<TS, SVR_ACT_EXPLIN>(kind, A, grid, s);
}

static hipError_t launch_render(RKind kind, const RenderArgs& A, const svr_opts& o, const Layout& L,
                                void* ws, hipStream_t s) {
  if (L.T == 0) return hipSuccess;
  unsigned grid;
  if (L.persistent > 0) {
    hipError_t e = launch_fill_u32(at<WsHeader>(ws, L.hdr)->work, 0u, 8, s);
    if (e != hipSuccess) return e;
    grid = (unsigned)min((int64_t)L.persistent, (int64_t)L.T + A.max_split);
  } else {
    grid = (unsigned)L.T + (kind == RKind::kBwd ? (unsigned)A.split_wgs : 0u);
  }
  switch (L.tile) {
    case 8: launch_act<8>(kind, A, o.activation, grid, s); break;
    case 32: launch_act<32>(kind, A, o.activation, grid, s); break;
    default: launch_act<16>(kind, A, o.activation, grid, s); break;
  }
  return hipGetLastError();
}

hipError_t launch_render_fwd(const svr_scene& sc, const CamSet& cams, const svr_opts& o,
                             const Layout& L, void* ws, const uint32_t* vals, float* rgba,
                             const svr_extra* extra, hipStream_t s) {
  (void)sc;
  RenderArgs A = render_args(cams, o, L, ws, vals);
  A.rgba = reinterpret_cast<float4*>(rgba);
  if (extra) {
    A.max_weight = reinterpret_cast<uint32_t*>(extra->max_weight);
    A.depth = extra->depth;
    A.normal = extra->normal;
    A.aux = (extra->depth || extra->normal) ? 1 : 0;
  }
  return launch_render(RKind::kFwd, A, o, L, ws, s);
}

hipError_t launch_render_stats(const svr_scene& sc, const CamSet& cams, const svr_opts& o,
                               const Layout& L, void* ws, const uint32_t* vals, hipStream_t s) {
  (void)sc;
  hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t*>(at<WsHeader>(ws, L.hdr)->stats), 0u,
                                 6, s);
  if (e != hipSuccess) return e;
  RenderArgs A = render_args(cams, o, L, ws, vals);
  return launch_render(RKind::kStats, A, o, L, ws, s);
}

hipError_t launch_render_bwd(const svr_scene& sc, const CamSet& cams, const svr_opts& o,
                             const Layout& L, void* ws, const uint32_t* vals,
                             const float* grad_rgba, const svr_extra* extra, hipStream_t s) {
  (void)sc;
  RenderArgs A = render_args(cams, o, L, ws, vals);
  A.grad_rgba = reinterpret_cast<const float4*>(grad_rgba);
  if (extra) {
    A.priority = extra->priority;
    A.grad_depth = extra->grad_depth;
    A.grad_normal = extra->grad_normal;
    A.aux = (extra->grad_depth || extra->grad_normal) ? 1 : 0;
  }
  FillSet z;
  z.add(at<uint32_t>(ws, L.g_corner), L.N * 8);
  z.add(at<uint32_t>(ws, L.g_rgb), L.NV * 3);
  if (A.aux) z.add(at<uint32_t>(ws, L.g_nrm), L.N * 3);
  hipError_t e = launch_zero_u32(z, s);
  if (e != hipSuccess) return e;
  return launch_render(RKind::kBwd, A, o, L, ws, s);
}

// grad_grid[m] = sum of the corner gradients of the corner slots sharing grid
// point m, in the adjacency's fixed order (no atomics)
__global__ __launch_bounds__(kBlock) void k_grid_gather(int64_t M, const int32_t* __restrict__ off,
                                                        const int32_t* __restrict__ adj,
                                                        const float* __restrict__ g_corner,
                                                        float* __restrict__ grad_grid,
                                                        int accumulate) {
  // grid points of one XCD are contiguous: they share voxels, whose 8 corner
  // gradients sit in one 32-byte block, so that block is read once per L2
  const int64_t nb = (M + kBlock - 1) / kBlock;
  const int64_t m = xcd_block(blockIdx.x, nb) * kBlock + threadIdx.x;
  if (m >= M) return;
  // a grid point is a corner of at most 8 voxels: the slots are loaded
  // together, then their gradients, then summed in slot order
  const int32_t e0 = off[m], e1 = off[m + 1];
  float acc = 0.f;
  if (e1 - e0 <= 8) {
    int32_t a[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) a[k] = e0 + k < e1 ? adj[e0 + k] : -1;
    float g[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) g[k] = a[k] >= 0 ? g_corner[a[k]] : 0.f;
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if (e0 + k < e1) acc += g[k];
  } else {
    for (int32_t e = e0; e < e1; ++e) acc += g_corner[adj[e]];
  }
  grad_grid[m] = accumulate ? grad_grid[m] + acc : acc;
}

hipError_t launch_sh_bwd(const svr_scene& sc, const CamSet& cams, const Layout& L, void* ws,
                         float* grad_grid, float* grad_sh, bool accumulate, bool aux,
                         hipStream_t s) {
  const bool gather = sc.grid_adj_off != nullptr && sc.grid_adj != nullptr;
  if (grad_grid && !accumulate && !gather) {
    hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t*>(grad_grid), 0u, sc.n_grid, s);
    if (e != hipSuccess) return e;
  }
  if (L.N > 0) {
    const dim3 grid((unsigned)((L.N + kBlock - 1) / kBlock));
#define SVR_SHB(D)                                                                             \
  SVR_LAUNCH("sh_bwd", k_sh_bwd<D>, grid, dim3(kBlock), 0, s, L.N, L.n_cams, cams, sc.center,   \
             sc.vox_grid, at<uint32_t>(ws, L.count), at<VoxRec>(ws, L.rec),                     \
             at<float>(ws, L.g_rgb), at<float>(ws, L.g_corner), grad_grid, grad_sh,            \
             sc.grid_raw, aux ? at<float>(ws, L.g_nrm) : nullptr, accumulate ? 1 : 0,          \
             gather ? 0 : 1, (reinterpret_cast<uintptr_t>(grad_sh) & 15u) == 0u ? 1 : 0)
    switch (sc.sh_degree) {
      case 0: SVR_SHB(0); break;
      case 1: SVR_SHB(1); break;
      case 2: SVR_SHB(2); break;
      default: SVR_SHB(3); break;
    }
#undef SVR_SHB
  }
  if (grad_grid && gather && sc.n_grid > 0) {
    const int64_t nb = (sc.n_grid + kBlock - 1) / kBlock;
    SVR_LAUNCH("grid_gather", k_grid_gather, dim3((unsigned)(((nb + 7) >> 3) << 3)),
               dim3(kBlock), 0, s, sc.n_grid, sc.grid_adj_off, sc.grid_adj,
               at<float>(ws, L.g_corner), grad_grid, accumulate ? 1 : 0);
  }
  return hipGetLastError();
}

}  // namespace svr
