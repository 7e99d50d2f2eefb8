// Sparse-voxel TSDF fusion and marching cubes (Sec. 3.2.4 "Sparse-voxel
// TSDF Fusion and Marching Cubes").
//
//   k_tsdf_fuse    one thread per grid point: for every camera, project the
//                  point (fp64), take the depth of the pixel whose square
//                  holds the projection (the composited depth divided by
//                  the pixel's opacity when the rgba image is given, no
//                  depth below the opacity threshold) and the signed
//                  distance along that ray, sdf = depth - |p - o|; observations with
//                  sdf >= -trunc add min(sdf / trunc, 1) with weight 1; the
//                  value is their mean (1 with weight 0 when never seen).
//   k_mesh_cells   one thread per voxel (one cell, its 8 corner grid
//                  points): the cell's case (corners above the iso value)
//                  selects up to kMaxCellTris triangles from a table built at
//                  compile time; each vertex sits on a cell edge, is keyed by
//                  that edge's two grid points (so neighbouring cells share
//                  it) and placed by linear interpolation.  A workgroup
//                  reserves the triangles of its voxels with one atomic.
//
// The table follows one rule per cell: on each face the crossing edges are
// paired (two crossings: one segment; four: two segments, each cutting off
// one above corner), every segment oriented with the above corners on its
// left seen from outside the cell; the segments chain into loops whose
// right-hand normal points towards increasing values; each loop starts at
// its crossing edge with the smallest corner pair (8 a + b, a < b) and is
// cut into a fan from there.
#include "svr_internal.h"

namespace svr {

constexpr int kMaxCellTris = 12;

struct MeshTable {
  uint8_t n[256];                      // triangles per case
  uint8_t v[256][kMaxCellTris * 3];    // vertices: corner pair a << 3 | b, a < b
};

constexpr MeshTable build_mesh_table() {
  MeshTable t{};
  // doubled unit-cell corner coordinates of corner c = 4x + 2y + z
  auto cx = [](int c) { return 2 * ((c >> 2) & 1); };
  auto cy = [](int c) { return 2 * ((c >> 1) & 1); };
  auto cz = [](int c) { return 2 * (c & 1); };
  for (int cs = 0; cs < 256; ++cs) {
    int nxt[64] = {};
    for (int i = 0; i < 64; ++i) nxt[i] = -1;
    for (int axis = 0; axis < 3; ++axis) {
      const int bit = axis == 0 ? 4 : (axis == 1 ? 2 : 1);
      const int o1 = axis == 0 ? 2 : 4, o2 = axis == 2 ? 2 : 1;
      for (int side = 0; side < 2; ++side) {
        const int base = side ? bit : 0;
        const int ring[4] = {base, base | o1, base | o1 | o2, base | o2};
        int nrm[3] = {0, 0, 0};
        nrm[axis] = side ? 1 : -1;
        bool up[4] = {};
        for (int i = 0; i < 4; ++i) up[i] = (cs >> ring[i]) & 1;
        int cross[4] = {}, nc = 0;
        for (int i = 0; i < 4; ++i)
          if (up[i] != up[(i + 1) & 3]) cross[nc++] = i;
        int seg_i[2] = {}, seg_j[2] = {}, seg_c[2] = {}, ns = 0;
        if (nc == 2) {
          int above_corner = -1;
          for (int i = 0; i < 4 && above_corner < 0; ++i)
            if (up[i]) above_corner = ring[i];
          seg_i[0] = cross[0];
          seg_j[0] = cross[1];
          seg_c[0] = above_corner;
          ns = 1;
        } else if (nc == 4) {
          for (int j = 0; j < 4; ++j)
            if (up[j]) {
              seg_i[ns] = (j + 3) & 3;
              seg_j[ns] = j;
              seg_c[ns] = ring[j];
              ++ns;
            }
        }
        for (int s = 0; s < ns; ++s) {
          int a0 = ring[seg_i[s]], b0 = ring[(seg_i[s] + 1) & 3];
          int a1 = ring[seg_j[s]], b1 = ring[(seg_j[s] + 1) & 3];
          if (a0 > b0) { const int q = a0; a0 = b0; b0 = q; }
          if (a1 > b1) { const int q = a1; a1 = b1; b1 = q; }
          // doubled edge midpoints, direction between them and the corner
          const int m0[3] = {(cx(a0) + cx(b0)) / 2, (cy(a0) + cy(b0)) / 2, (cz(a0) + cz(b0)) / 2};
          const int m1[3] = {(cx(a1) + cx(b1)) / 2, (cy(a1) + cy(b1)) / 2, (cz(a1) + cz(b1)) / 2};
          const int d[3] = {m1[0] - m0[0], m1[1] - m0[1], m1[2] - m0[2]};
          const int q[3] = {cx(seg_c[s]) - m0[0], cy(seg_c[s]) - m0[1], cz(seg_c[s]) - m0[2]};
          // left of d seen from outside: nrm x d
          const int l[3] = {nrm[1] * d[2] - nrm[2] * d[1], nrm[2] * d[0] - nrm[0] * d[2],
                            nrm[0] * d[1] - nrm[1] * d[0]};
          const int dot = l[0] * q[0] + l[1] * q[1] + l[2] * q[2];
          const int e0 = a0 * 8 + b0, e1 = a1 * 8 + b1;
          if (dot > 0) nxt[e0] = e1;
          else nxt[e1] = e0;
        }
      }
    }
    // loops in increasing order of their first (smallest) corner pair
    bool seen[64] = {};
    int nt = 0;
    for (int e0 = 0; e0 < 64; ++e0) {
      if (nxt[e0] < 0 || seen[e0]) continue;
      int loop[12] = {}, len = 0;
      int e = e0;
      do {
        loop[len++] = e;
        seen[e] = true;
        e = nxt[e];
      } while (e != e0 && len < 12);
      for (int i = 1; i + 1 < len; ++i) {
        t.v[cs][3 * nt + 0] = (uint8_t)loop[0];
        t.v[cs][3 * nt + 1] = (uint8_t)loop[i];
        t.v[cs][3 * nt + 2] = (uint8_t)loop[i + 1];
        ++nt;
      }
    }
    t.n[cs] = (uint8_t)nt;
  }
  return t;
}

__constant__ MeshTable kMesh = build_mesh_table();
constexpr MeshTable kMeshHost = build_mesh_table();

void mesh_case_table(uint8_t* counts, uint8_t* verts) {
  for (int c = 0; c < 256; ++c) {
    counts[c] = kMeshHost.n[c];
    for (int j = 0; j < kMaxCellTris * 3; ++j) verts[c * kMaxCellTris * 3 + j] = kMeshHost.v[c][j];
  }
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_tsdf_fuse(int64_t M, const float* __restrict__ gp,
                                                      FuseCamSet cams,
                                                      const float* __restrict__ depth,
                                                      const float* __restrict__ rgba,
                                                      float min_alpha, float trunc,
                                                      float* __restrict__ tsdf,
                                                      float* __restrict__ weight,
                                                      const uint32_t* __restrict__ order,
                                                      int first, int last) {
  // contiguous grid points per XCD: spatial neighbours when the visit order
  // is, whose projections fall on the same image lines, read once per L2
  const int64_t nb = (M + kBlock - 1) / kBlock;
  const int64_t i = xcd_block(blockIdx.x, nb) * kBlock + threadIdx.x;
  if (i >= M) return;
  // visit order (a Morton order keeps a wave's projections on few image lines)
  const int64_t m = order ? (int64_t)order[i] : i;
  if (m >= M) return;  // not a permutation entry
  const double px = gp[m], py = gp[M + m], pz = gp[2 * M + m];
  // between camera groups tsdf holds the running sum of the added values
  float acc = first ? 0.f : tsdf[m], w = first ? 0.f : weight[m];
  for (int ci = 0; ci < cams.n; ++ci) {
    const FuseCam& c = cams.c[ci];
    const double z = (double)c.r[6] * px + (double)c.r[7] * py + (double)c.r[8] * pz + (double)c.t[2];
    if (!(z > 0.0)) continue;
    const double x = (double)c.r[0] * px + (double)c.r[1] * py + (double)c.r[2] * pz + (double)c.t[0];
    const double y = (double)c.r[3] * px + (double)c.r[4] * py + (double)c.r[5] * pz + (double)c.t[1];
    const double u = (double)c.fx * x / z + (double)c.cx;
    const double v = (double)c.fy * y / z + (double)c.cy;
    const double fu = floor(u), fv = floor(v);
    if (!(fu >= 0.0 && fu < (double)c.W && fv >= 0.0 && fv < (double)c.H)) continue;
    const int64_t pix = c.pix_off + (int64_t)fv * c.W + (int64_t)fu;
    float d = depth[pix];
    if (rgba && d > 0.f) {  // d <= 0 gives no depth either way
      const float a = rgba[4 * pix + 3];
      d = (a >= min_alpha && a > 0.f) ? d / a : 0.f;
    }
    if (!(d > 0.f)) continue;
    const double rx = px - c.od[0], ry = py - c.od[1], rz = pz - c.od[2];
    const double sdf = (double)d - sqrt(rx * rx + ry * ry + rz * rz);
    if (sdf < -(double)trunc) continue;
    acc += (float)fmin(sdf / (double)trunc, 1.0);
    w += 1.f;
  }
  tsdf[m] = last ? (w > 0.f ? acc / w : 1.f) : acc;
  weight[m] = w;
}

// Voxels per thread of the cell kernel: a workgroup covers kBlock * kCellsPer
// consecutive voxels and reserves their triangles with one atomic.
constexpr int kCellsPer = 4;

__device__ __forceinline__ int cell_case(int64_t v, int64_t N, const int32_t* __restrict__ vox_grid,
                                         const float* __restrict__ field,
                                         const float* __restrict__ weight, float iso, int* g,
                                         float* f, uint32_t& cs) {
  cs = 0;
  if (v >= N) return 0;
  const int4* vg = reinterpret_cast<const int4*>(vox_grid + v * 8);
  const int4 ga = vg[0], gb = vg[1];
  g[0] = ga.x; g[1] = ga.y; g[2] = ga.z; g[3] = ga.w;
  g[4] = gb.x; g[5] = gb.y; g[6] = gb.z; g[7] = gb.w;
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    f[c] = field[g[c]];
    cs |= (f[c] > iso ? 1u : 0u) << c;
  }
  const int n = (int)kMesh.n[cs];
  if (n == 0 || !weight) return n;
  // weights only matter where the surface crosses the cell
  bool ok = true;
#pragma unroll
  for (int c = 0; c < 8; ++c) ok &= weight[g[c]] != 0.f;
  return ok ? n : 0;
}

__global__ __launch_bounds__(kBlock) void k_mesh_cells(
    int64_t N, const float* __restrict__ center, const float* __restrict__ size,
    const int32_t* __restrict__ vox_grid, const float* __restrict__ field,
    const float* __restrict__ weight, float iso, int64_t max_tris, int32_t* __restrict__ keys,
    float* __restrict__ pos, unsigned long long* __restrict__ count,
    const uint32_t* __restrict__ order) {
  __shared__ int s_wave[kBlock / 64];
  __shared__ unsigned long long s_base;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int64_t v0 = (int64_t)blockIdx.x * kBlock * kCellsPer + threadIdx.x;
  int g[kCellsPer][8];
  float f[kCellsPer][8];
  uint32_t cs[kCellsPer];
  int nt[kCellsPer];
  int64_t vr[kCellsPer];
  int mine = 0;
#pragma unroll
  for (int r = 0; r < kCellsPer; ++r) {
    const int64_t i = v0 + (int64_t)r * kBlock;
    vr[r] = (order && i < N) ? (int64_t)order[i] : i;  // visit order
    nt[r] = cell_case(vr[r], N, vox_grid, field, weight, iso, g[r], f[r], cs[r]);
    mine += nt[r];
  }
  // workgroup exclusive scan of the per-thread triangle counts
  int incl = mine;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int q = __shfl_up(incl, o, 64);
    if (lane >= o) incl += q;
  }
  if (lane == 63) s_wave[wid] = incl;
  __syncthreads();
  int before = 0, total = 0;
#pragma unroll
  for (int w = 0; w < kBlock / 64; ++w) {
    const int t = s_wave[w];
    before += w < wid ? t : 0;
    total += t;
  }
  if (total == 0) return;  // uniform over the workgroup
  if (threadIdx.x == 0) s_base = atomicAdd(count, (unsigned long long)total);
  __syncthreads();
  unsigned long long first = s_base + (unsigned long long)(before + incl - mine);
#pragma unroll
  for (int r = 0; r < kCellsPer; ++r) {
    const int n = nt[r];
    if (n == 0) continue;
    const unsigned long long at = first;
    first += (unsigned long long)n;
    if (at + (unsigned long long)n > (unsigned long long)max_tris) continue;  // caller sees count
    const int64_t v = vr[r];
    const float s = size[v];
    const float ox = center[v] - 0.5f * s, oy = center[N + v] - 0.5f * s,
                oz = center[2 * N + v] - 0.5f * s;
    for (int k = 0; k < n; ++k) {
      const int64_t tri = (int64_t)(at + (unsigned long long)k);
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const int code = kMesh.v[cs[r]][3 * k + j];
        const int a = code >> 3, b = code & 7;
        const float t = (iso - f[r][a]) / (f[r][b] - f[r][a]);
        const float ax = ox + s * (float)((a >> 2) & 1), ay = oy + s * (float)((a >> 1) & 1),
                    az = oz + s * (float)(a & 1);
        const float bx = ox + s * (float)((b >> 2) & 1), by = oy + s * (float)((b >> 1) & 1),
                    bz = oz + s * (float)(b & 1);
        pos[tri * 9 + 3 * j + 0] = ax + t * (bx - ax);
        pos[tri * 9 + 3 * j + 1] = ay + t * (by - ay);
        pos[tri * 9 + 3 * j + 2] = az + t * (bz - az);
        keys[tri * 6 + 2 * j + 0] = min(g[r][a], g[r][b]);
        keys[tri * 6 + 2 * j + 1] = max(g[r][a], g[r][b]);
      }
    }
  }
}

// 10 bits of a coordinate spread to every third bit
__device__ __forceinline__ uint64_t spread3(uint32_t x) {
  uint64_t v = x & 0x3ffu;
  v = (v | (v << 16)) & 0x30000ffull;
  v = (v | (v << 8)) & 0x300f00full;
  v = (v | (v << 4)) & 0x30c30c3ull;
  v = (v | (v << 2)) & 0x9249249ull;
  return v;
}

__global__ __launch_bounds__(kBlock) void k_morton_keys(int64_t n, const float* __restrict__ pos,
                                                        float lx, float ly, float lz, float inv,
                                                        uint64_t* __restrict__ keys,
                                                        uint32_t* __restrict__ vals) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const float q[3] = {(pos[i] - lx) * inv, (pos[n + i] - ly) * inv, (pos[2 * n + i] - lz) * inv};
  uint32_t c[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float t = fminf(fmaxf(q[a], 0.f), 1023.f);  // NaN -> 0
    c[a] = (uint32_t)t;
  }
  keys[i] = spread3(c[0]) << 2 | spread3(c[1]) << 1 | spread3(c[2]);
  vals[i] = (uint32_t)i;
}

hipError_t launch_morton_keys(const float* pos, int64_t n, const float* lo, float extent,
                              uint64_t* keys, uint32_t* vals, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  SVR_LAUNCH("morton_keys", k_morton_keys, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock),
             0, s, n, pos, lo[0], lo[1], lo[2], 1024.f / extent, keys, vals);
  return hipGetLastError();
}

hipError_t launch_tsdf_fuse(const float* grid_pos, int64_t M, const FuseCamSet& cams, const float* depth,
                            const float* rgba, float min_alpha, float trunc, float* tsdf,
                            float* weight, const uint32_t* order, bool first, bool last,
                            hipStream_t s) {
  if (M <= 0) return hipSuccess;
  const int64_t nb = (M + kBlock - 1) / kBlock;
  SVR_LAUNCH("tsdf_fuse", k_tsdf_fuse, dim3((unsigned)(((nb + 7) >> 3) << 3)), dim3(kBlock), 0, s,
             M, grid_pos, cams, depth, rgba, min_alpha, trunc, tsdf, weight, order, first ? 1 : 0,
             last ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_mesh_cells(const svr_scene& sc, const float* field, const float* weight, float iso,
                             int64_t max_tris, int32_t* keys, float* pos, unsigned long long* count,
                             const uint32_t* order, hipStream_t s) {
  hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t*>(count), 0u, 2, s);
  if (e != hipSuccess || sc.n_voxels == 0) return e;
  const int64_t per = (int64_t)kBlock * kCellsPer;
  SVR_LAUNCH("mesh_cells", k_mesh_cells, dim3((unsigned)((sc.n_voxels + per - 1) / per)),
             dim3(kBlock), 0, s, sc.n_voxels, sc.center, sc.size, sc.vox_grid, field, weight, iso,
             max_tris, keys, pos, count, order);
  return hipGetLastError();
}

}  // namespace svr
