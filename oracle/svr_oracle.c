/*
 * svr_oracle.c -- FP64 CPU reference ("oracle") for the sparse-voxel
 * rasterizer of "Sparse Voxels Rasterization" (Sun et al., CVPR 2025,
 * arXiv 2412.04459).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file; only the tests, the smoke check and the CPU leg of the
 * benchmark do.  It shares no code with the GPU library: every formula here
 * is written out again from the paper.
 *
 * What it computes is the plain definition the rasterizer is an acceleration
 * of: for every pixel ray, intersect EVERY voxel box, order the hits by their
 * entry distance, and alpha-composite them front to back (Sec. 3.1, eq.
 * alpha_blend; Sec. 3.1.2 "Rendering pixels").  The proof of Supp. B.3 says
 * the tile/Morton sort reaches exactly this order, so no tiles and no sort
 * keys enter the image or gradient computation.
 *
 * All scene parameters are taken in double precision (callers promote the
 * fp32 scene exactly), so finite differences can be taken in FP64.
 *
 * Readings taken where the paper is silent (each documented in the design
 * notes):
 *   - voxel centre and size are given per voxel;
 *   - camera: OpenCV pinhole, pixel centres at +0.5, unit ray direction;
 *   - a voxel is composited iff the transmittance BEFORE it is >= t_stop;
 *   - output is premultiplied RGB plus A = 1 - T_final;
 *   - SH: real spherical harmonics up to degree 3, index l*l + l + m,
 *     normalisation N_lm (x sqrt 2 for m != 0), no Condon-Shortley phase;
 *     colour = max(0, sum) with no offset;
 *   - softplus with beta = 1.
 *
 * Parity pins live in the tests (closed forms, brute force, finite
 * differences, the paper's printed order tables).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_MAX_LEVELS 16

/* ------------------------------------------------------------------------ */
/* camera: cam[0..5] = W, H, fx, fy, cx, cy; cam[6..17] = w2c row-major 3x4   */
/* ------------------------------------------------------------------------ */
static void cam_origin(const double* cam, double o[3]) {
  const double* M = cam + 6;
  /* o = -R^T t */
  for (int c = 0; c < 3; ++c)
    o[c] = -(M[0 * 4 + c] * M[3] + M[1 * 4 + c] * M[7] + M[2 * 4 + c] * M[11]);
}

/* un-normalised world direction through the centre of pixel (u, v) */
static void cam_dir_raw(const double* cam, int u, int v, double d[3]) {
  const double* M = cam + 6;
  double dc[3] = {((double)u + 0.5 - cam[4]) / cam[2], ((double)v + 0.5 - cam[5]) / cam[3], 1.0};
  for (int c = 0; c < 3; ++c) d[c] = M[0 * 4 + c] * dc[0] + M[1 * 4 + c] * dc[1] + M[2 * 4 + c] * dc[2];
}

static void normalize3(double d[3]) {
  double n = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  d[0] /= n; d[1] /= n; d[2] /= n;
}

/* ------------------------------------------------------------------------ */
/* activation (Sec. 3.1.1 eq. explin; softplus as the alternative)           */
/* ------------------------------------------------------------------------ */
double oracle_act(double x, int act) {
  if (act == 0) {
    if (x > 1.1) return x;
    return exp(x / 1.1 - 1.0 + log(1.1));
  }
  /* softplus, beta = 1, evaluated stably */
  if (x > 0) return x + log1p(exp(-x));
  return log1p(exp(x));
}

double oracle_act_grad(double x, int act) {
  if (act == 0) {
    if (x > 1.1) return 1.0;
    return exp(x / 1.1 - 1.0 + log(1.1)) / 1.1;
  }
  /* d/dx softplus = logistic(x) */
  if (x >= 0) return 1.0 / (1.0 + exp(-x));
  double e = exp(x);
  return e / (1.0 + e);
}

/* ------------------------------------------------------------------------ */
/* real spherical harmonics via associated Legendre functions (Sec. 3.1.1    */
/* eq. vox_color uses an SH evaluation; the basis is not printed, so the     */
/* textbook real basis is used):                                             */
/*   Y_l0 = N_l0 P_l(cos t),                                                 */
/*   Y_lm = sqrt2 N_lm P_l^m(cos t) cos(m phi),   m > 0                      */
/*   Y_l-m = sqrt2 N_lm P_l^m(cos t) sin(m phi),  m > 0                      */
/*   N_lm = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!), P_l^m without (-1)^m.        */
/* ------------------------------------------------------------------------ */
static double factorial(int n) { double f = 1; for (int i = 2; i <= n; ++i) f *= i; return f; }

static double assoc_legendre(int l, int m, double x) {
  /* P_m^m = (2m-1)!! (1-x^2)^(m/2) */
  double pmm = 1.0;
  double sx = sqrt(fmax(0.0, 1.0 - x * x));
  for (int i = 1; i <= m; ++i) pmm *= (2.0 * i - 1.0) * sx;
  if (l == m) return pmm;
  double pm1 = x * (2.0 * m + 1.0) * pmm;
  if (l == m + 1) return pm1;
  double pl = 0;
  for (int ll = m + 2; ll <= l; ++ll) {
    pl = ((2.0 * ll - 1.0) * x * pm1 - (ll + m - 1.0) * pmm) / (double)(ll - m);
    pmm = pm1;
    pm1 = pl;
  }
  return pl;
}

void oracle_sh_basis(int degree, const double dir_in[3], double* Y) {
  double d[3] = {dir_in[0], dir_in[1], dir_in[2]};
  normalize3(d);
  double ct = d[2];
  double phi = atan2(d[1], d[0]);
  for (int l = 0; l <= degree; ++l) {
    for (int m = -l; m <= l; ++m) {
      int am = m < 0 ? -m : m;
      double N = sqrt((2.0 * l + 1.0) / (4.0 * M_PI) * factorial(l - am) / factorial(l + am));
      double P = assoc_legendre(l, am, ct);
      double y;
      if (m == 0) y = N * P;
      else if (m > 0) y = sqrt(2.0) * N * P * cos(am * phi);
      else y = sqrt(2.0) * N * P * sin(am * phi);
      Y[l * l + l + m] = y;
    }
  }
}

/* ------------------------------------------------------------------------ */
/* octree path <-> voxel index (Supp. A.1).  A voxel of level lv has integer  */
/* index (i, j, k) in [0, 2^lv)^3 among the cells of its level.  Descending   */
/* from the root, the ancestor of level l has index (i, j, k) >> (lv - l),    */
/* and the child taken at level l is the low bit of that ancestor index on    */
/* each axis: octant 4x + 2y + z.  The path stores the octant of level l at   */
/* bits 3(16 - l) .. 3(16 - l) + 2 (coarsest level highest, unused levels 0). */
/* ------------------------------------------------------------------------ */
uint64_t oracle_to_octpath(int64_t i, int64_t j, int64_t k, int lv) {
  uint64_t path = 0;
  for (int l = 1; l <= lv; ++l) {
    int sh = lv - l; /* the ancestor of level l drops the sh finest index bits */
    int ox = (int)((i >> sh) & 1), oy = (int)((j >> sh) & 1), oz = (int)((k >> sh) & 1);
    uint64_t octant = (uint64_t)(4 * ox + 2 * oy + oz);
    path |= octant << (3 * (OR_MAX_LEVELS - l));
  }
  return path;
}

/* inverse: walk the path from the root, doubling the index at every level   */
/* and adding the child's bit on each axis                                   */
void oracle_to_voxel_index(uint64_t path, int lv, int64_t out[3]) {
  int64_t idx[3] = {0, 0, 0};
  for (int l = 1; l <= lv; ++l) {
    int octant = (int)((path >> (3 * (OR_MAX_LEVELS - l))) & 7);
    for (int ax = 0; ax < 3; ++ax) idx[ax] = 2 * idx[ax] + ((octant >> (2 - ax)) & 1);
  }
  out[0] = idx[0]; out[1] = idx[1]; out[2] = idx[2];
}

/* ------------------------------------------------------------------------ */
/* direction-dependent Morton order (Supp. B.2)                              */
/* For ray sign bits s (bit 2: d_x < 0, bit 1: d_y < 0, bit 0: d_z < 0) the  */
/* eight children of a node are visited near side first on every axis: on an */
/* axis the ray travels along +, the low child (bit 0) is nearer; on an axis */
/* it travels along -, the high child is nearer.  The rank of child t is     */
/* therefore built axis by axis.  The permutation is applied to all 16       */
/* triplets of the path, coarsest level in the top triplet.                  */
/* ------------------------------------------------------------------------ */
int oracle_child_rank(int s, int t) {
  int r = 0;
  for (int ax = 0; ax < 3; ++ax) {
    int bit = (t >> (2 - ax)) & 1;
    int neg = (s >> (2 - ax)) & 1;
    int near_first = neg ? (1 - bit) : bit;
    r |= near_first << (2 - ax);
  }
  return r;
}

uint64_t oracle_morton_order(uint64_t octpath, int s) {
  uint64_t order = 0;
  for (int n = 0; n < OR_MAX_LEVELS; ++n) {
    int t = (int)((octpath >> (3 * n)) & 7);
    order |= (uint64_t)oracle_child_rank(s, t) << (3 * n);
  }
  return order;
}

/* Sort keys and values for given (tile, voxel, s) triples.
 *   paper form (Supp. B.1): key = tile << 48 | order, value = s << 29 | vid.
 *   compact form (same order within and across tiles whenever
 *   max_level <= 15, because the 3*(16-max_level) low bits of the order are
 *   copies of s): key = tile << (3 max_level + 3) | order_top << 3 | s.       */
void oracle_keys(int64_t n, const int64_t* tile, const int64_t* vid, const uint8_t* s,
                 const uint64_t* octpath, int max_level, uint64_t* key_paper,
                 uint64_t* key_compact, uint32_t* value) {
  for (int64_t e = 0; e < n; ++e) {
    uint64_t order = oracle_morton_order(octpath[vid[e]], s[e]);
    if (key_paper) key_paper[e] = ((uint64_t)tile[e] << 48) | order;
    if (key_compact) {
      uint64_t top = order >> (3 * (OR_MAX_LEVELS - max_level));
      key_compact[e] = ((uint64_t)tile[e] << (3 * max_level + 3)) | (top << 3) | (uint64_t)s[e];
    }
    if (value) value[e] = ((uint32_t)s[e] << 29) | (uint32_t)vid[e];
  }
}

/* ------------------------------------------------------------------------ */
/* ray / axis-aligned box (Supp. A.2, the ray-box test): the points o + t d  */
/* inside the box [c - s/2, c + s/2]^3 form one interval of t, the           */
/* intersection over the three axes of the interval between that axis'      */
/* two bounding planes (empty if the ray runs parallel to the planes outside */
/* them, unbounded if inside).  a is where the ray enters the box, b where   */
/* it leaves.  The voxel is hit iff the interval is non-empty and starts in  */
/* front of the camera, a > 0 (so a camera inside a voxel skips it).         */
/* ------------------------------------------------------------------------ */
static int ray_aabb(const double c[3], double s, const double o[3], const double d[3],
                    double* a_out, double* b_out) {
  double enter = -INFINITY, leave = INFINITY;
  for (int ax = 0; ax < 3; ++ax) {
    double lo = c[ax] - 0.5 * s, hi = c[ax] + 0.5 * s;
    double t_lo, t_hi; /* the part of the ray between the planes x_ax = lo and x_ax = hi */
    if (d[ax] > 0) {
      t_lo = (lo - o[ax]) / d[ax];
      t_hi = (hi - o[ax]) / d[ax];
    } else if (d[ax] < 0) {
      t_lo = (hi - o[ax]) / d[ax];
      t_hi = (lo - o[ax]) / d[ax];
    } else if (o[ax] >= lo && o[ax] <= hi) {
      t_lo = -INFINITY;
      t_hi = INFINITY;
    } else {
      t_lo = INFINITY;
      t_hi = -INFINITY;
    }
    if (t_lo > enter) enter = t_lo;
    if (t_hi < leave) leave = t_hi;
  }
  *a_out = enter;
  *b_out = leave;
  return (enter <= leave) && (enter > 0);
}

/* trilinear weights of the 8 corners (Supp. A.2 eq. interp; corner index     */
/* c = 4 x + 2 y + z)                                                          */
static void trilinear_weights(const double q[3], double w[8]) {
  for (int c = 0; c < 8; ++c) {
    double wx = ((c >> 2) & 1) ? q[0] : 1.0 - q[0];
    double wy = ((c >> 1) & 1) ? q[1] : 1.0 - q[1];
    double wz = (c & 1) ? q[2] : 1.0 - q[2];
    w[c] = wx * wy * wz;
  }
}

typedef struct {
  double a, b;
  int64_t id;
} hit_t;

static int hit_cmp(const void* pa, const void* pb) {
  const hit_t* x = (const hit_t*)pa;
  const hit_t* y = (const hit_t*)pb;
  if (x->a < y->a) return -1;
  if (x->a > y->a) return 1;
  return (x->id < y->id) ? -1 : (x->id > y->id);
}

typedef struct {
  int64_t N;
  const double* center; /* [3][N] */
  const double* size;
  const int32_t* vox_grid; /* [N][8] */
  const double* grid_raw;
  const double* sh; /* [N][nb][3] */
  int sh_degree;
} scene_t;

/* colour of voxel i seen from o (Sec. 3.1.1 eq. vox_color), and the SH     */
/* basis used (for the adjoint); pre is the value before the clamp          */
static void voxel_color(const scene_t* S, int64_t i, const double o[3], double rgb[3],
                        double pre[3], double* Y) {
  double dir[3];
  for (int ax = 0; ax < 3; ++ax) dir[ax] = S->center[ax * S->N + i] - o[ax];
  oracle_sh_basis(S->sh_degree, dir, Y);
  int nb = (S->sh_degree + 1) * (S->sh_degree + 1);
  for (int ch = 0; ch < 3; ++ch) {
    double acc = 0;
    for (int j = 0; j < nb; ++j) acc += S->sh[(i * nb + j) * 3 + ch] * Y[j];
    pre[ch] = acc;
    rgb[ch] = acc > 0 ? acc : 0;
  }
}

/* optical depth x = (l/K) sum_k act(v_k) of the segment [a,b] through voxel */
/* i (Sec. 3.1.1 eq. vox_alpha, Supp. A.2 eq. K_samp_pts); optionally also  */
/* dx/dV for the 8 corner raw densities                                      */
static double segment_depth(const scene_t* S, int64_t i, const double o[3], const double d[3],
                            double a, double b, int K, int act, double dxdV[8]) {
  double c[3], s = S->size[i];
  for (int ax = 0; ax < 3; ++ax) c[ax] = S->center[ax * S->N + i];
  double V[8];
  for (int k = 0; k < 8; ++k) V[k] = S->grid_raw[S->vox_grid[i * 8 + k]];
  double dn = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  double l = (b - a) * dn;
  double sum = 0;
  if (dxdV) for (int k = 0; k < 8; ++k) dxdV[k] = 0;
  for (int k = 1; k <= K; ++k) {
    double t = a + ((double)k - 0.5) / (double)K * (b - a);
    double q[3], w[8];
    for (int ax = 0; ax < 3; ++ax) q[ax] = (o[ax] + t * d[ax] - (c[ax] - 0.5 * s)) / s;
    trilinear_weights(q, w);
    double v = 0;
    for (int m = 0; m < 8; ++m) v += w[m] * V[m];
    sum += oracle_act(v, act);
    if (dxdV) {
      double g = oracle_act_grad(v, act);
      for (int m = 0; m < 8; ++m) dxdV[m] += g * w[m] * l / (double)K;
    }
  }
  return l / (double)K * sum;
}

/* Voxel normal (Sec. 3.1.1 "Voxel normal"; Supp. "Details of Voxel Normal"):  */
/* the gradient of the trilinear raw-density field at the voxel centre,      */
/* g = 0.25 [ (V100+V101+V110+V111) - (V000+V001+V010+V011), ... ], normalised; */
/* zero when g = 0.  With dLdn != NULL, adds dL/dV for dL/dn = dLdn:          */
/* dn/dg = (I - n n^T) / |g| and dg_b/dV_ijk = 0.25 (2 bit_b - 1).            */
static void voxel_normal(const scene_t* S, int64_t i, double n[3], const double* dLdn,
                         double dLdV[8]) {
  double V[8];
  for (int k = 0; k < 8; ++k) V[k] = S->grid_raw[S->vox_grid[i * 8 + k]];
  /* corner index c = 4x + 2y + z: V_xyz = V[4x + 2y + z] */
  double g[3];
  g[0] = 0.25 * ((V[4] + V[5] + V[6] + V[7]) - (V[0] + V[1] + V[2] + V[3]));
  g[1] = 0.25 * ((V[2] + V[3] + V[6] + V[7]) - (V[0] + V[1] + V[4] + V[5]));
  g[2] = 0.25 * ((V[1] + V[3] + V[5] + V[7]) - (V[0] + V[2] + V[4] + V[6]));
  double len = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
  for (int a = 0; a < 3; ++a) n[a] = len > 0 ? g[a] / len : 0.0;
  if (!dLdn || !(len > 0)) return;
  double dLdg[3];
  double nd = n[0] * dLdn[0] + n[1] * dLdn[1] + n[2] * dLdn[2];
  for (int b = 0; b < 3; ++b) dLdg[b] = (dLdn[b] - n[b] * nd) / len;
  for (int c = 0; c < 8; ++c) {
    int bit[3] = {(c >> 2) & 1, (c >> 1) & 1, c & 1};
    for (int b = 0; b < 3; ++b) dLdV[c] += dLdg[b] * 0.25 * (2.0 * bit[b] - 1.0);
  }
}

/* Voxel depth (Sec. 3.1.1 "Voxel depth"; Supp. "Details of Voxel Depth"):     */
/* the K samples of the segment with their own alphas                          */
/*   alpha_k = 1 - exp(-(l/K) act(v_k)),  t_k = a + (k - 1/2)/K (b - a)        */
/* composited locally: d = sum_k prod_{j<k} (1 - alpha_j) alpha_k t_k.         */
/* With dddV != NULL also dd/dV for the 8 corner raw densities, through        */
/* dd/dalpha_k = P_k (t_k - E_{k+1}) (P_k the product before k, E_{k+1} the    */
/* depth of the samples after k composited from k+1 on) and                    */
/* dalpha_k/dv_k = (1 - alpha_k) (l/K) act'(v_k).                              */
#define OR_MAX_K 64
static double segment_local_depth(const scene_t* S, int64_t i, const double o[3],
                                  const double d[3], double a, double b, int K, int act,
                                  double dddV[8]) {
  double c[3], s = S->size[i];
  for (int ax = 0; ax < 3; ++ax) c[ax] = S->center[ax * S->N + i];
  double V[8];
  for (int k = 0; k < 8; ++k) V[k] = S->grid_raw[S->vox_grid[i * 8 + k]];
  double dn = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  double l = (b - a) * dn;
  double al[OR_MAX_K], tk[OR_MAX_K], ag[OR_MAX_K], w[OR_MAX_K][8];
  if (K > OR_MAX_K) K = OR_MAX_K;
  for (int k = 1; k <= K; ++k) {
    double t = a + ((double)k - 0.5) / (double)K * (b - a);
    double q[3];
    for (int ax = 0; ax < 3; ++ax) q[ax] = (o[ax] + t * d[ax] - (c[ax] - 0.5 * s)) / s;
    trilinear_weights(q, w[k - 1]);
    double v = 0;
    for (int m = 0; m < 8; ++m) v += w[k - 1][m] * V[m];
    al[k - 1] = 1.0 - exp(-l / (double)K * oracle_act(v, act));
    ag[k - 1] = oracle_act_grad(v, act);
    tk[k - 1] = t * dn;
  }
  double dep = 0, P = 1.0;
  for (int k = 0; k < K; ++k) {
    dep += P * al[k] * tk[k];
    P *= 1.0 - al[k];
  }
  if (dddV) {
    for (int m = 0; m < 8; ++m) dddV[m] = 0;
    /* E after sample k, walking back */
    double E = 0, Pk[OR_MAX_K];
    P = 1.0;
    for (int k = 0; k < K; ++k) { Pk[k] = P; P *= 1.0 - al[k]; }
    for (int k = K - 1; k >= 0; --k) {
      double dd_dal = Pk[k] * (tk[k] - E);
      double dal_dv = (1.0 - al[k]) * l / (double)K * ag[k];
      for (int m = 0; m < 8; ++m) dddV[m] += dd_dal * dal_dv * w[k][m];
      E = al[k] * tk[k] + (1.0 - al[k]) * E;
    }
  }
  return dep;
}

/* collect and order the hits of one ray */
static int64_t collect_hits(const scene_t* S, const double o[3], const double d[3], hit_t** buf,
                            int64_t* cap) {
  int64_t n = 0;
  for (int64_t i = 0; i < S->N; ++i) {
    double c[3] = {S->center[i], S->center[S->N + i], S->center[2 * S->N + i]};
    double a, b;
    if (ray_aabb(c, S->size[i], o, d, &a, &b)) {
      if (n == *cap) {
        *cap = *cap ? 2 * *cap : 256;
        *buf = (hit_t*)realloc(*buf, (size_t)*cap * sizeof(hit_t));
      }
      (*buf)[n].a = a;
      (*buf)[n].b = b;
      (*buf)[n].id = i;
      ++n;
    }
  }
  if (n > 1) qsort(*buf, (size_t)n, sizeof(hit_t), hit_cmp);
  return n;
}

/* record of one composited hit */
typedef struct {
  int64_t id;
  double w;     /* blending weight T_i alpha_i */
  double prio;  /* |alpha_i dL/dalpha_i| */
  double g[11]; /* dL/dV[8], dL/dc[3] */
  double pre[3];
  double Y[16];
} grec_t;

/*
 * Render the listed pixels.
 *   rgba[p*4+0..3]      premultiplied RGB and A = 1 - T_final
 *   rgba_alt[p*4..]     the result with the first early-stop decision that
 *                       lies within the relative band `band` of t_stop taken
 *                       the other way (equal to rgba when flags[p] == 0)
 *   flags[p]            bit 0: a stop decision fell in the band;
 *                       bit 1: two hits with positive length have entry
 *                       distances closer than 1e-9 (order ambiguous)
 *   ncomp[p]            number of composited voxels; nhit[p] hits in total
 *   seq[p*max_seq+...]  composited voxel ids in order (if seq != NULL)
 * With g_rgba != NULL also accumulates, in pixel order, dL/d grid_raw and
 * dL/d sh for L = sum_p <g_rgba[p], rgba[p]>.
 * Training statistics of Sec. 3.2.2 (NULL: not computed), per voxel over the
 * listed pixels' composited hits:
 *   max_weight[N]  max of the blending weight T_i alpha_i ("Pruning")
 *   priority[N]    sum of |alpha_i dL/dalpha_i| (eq. priority; needs g_rgba;
 *                  the loss here is the rgba term)
 * Depth and normal images (Sec. 3.1.1 "Voxel normal", "Voxel depth"; NULL:
 * not computed), plain rule:
 *   depth[p]       D = sum_i T_i d_i, d_i the voxel's locally composited
 *                  sample depth (ray distance)
 *   normal[p*3..]  N = sum_i T_i alpha_i n_i
 * and, with g_rgba != NULL, g_depth[p] / g_normal[p*3..] (NULL: zero) add
 * <g_depth, D> + <g_normal, N> to L.
 */
int oracle_render(int64_t N, const double* center, const double* size, const int32_t* vox_grid,
                  const double* grid_raw, int64_t M, const double* sh, int sh_degree,
                  const double* cam, int K, double t_stop, int act, double band, int64_t npix,
                  const int64_t* pix, double* rgba, double* rgba_alt, uint8_t* flags,
                  int32_t* ncomp, int32_t* nhit, int32_t* seq, int max_seq, const double* g_rgba,
                  double* grad_grid, double* grad_sh, double* max_weight, double* priority,
                  double* depth, double* normal, const double* g_depth, const double* g_normal,
                  int nthreads) {
  scene_t S = {N, center, size, vox_grid, grid_raw, sh, sh_degree};
  int W = (int)cam[0];
  int nb = (sh_degree + 1) * (sh_degree + 1);
  double o[3];
  cam_origin(cam, o);
  grec_t** recs = NULL;
  int64_t* nrec = NULL;
  if (!g_rgba) priority = NULL;
  if (g_rgba || max_weight) {
    recs = (grec_t**)calloc((size_t)npix, sizeof(grec_t*));
    nrec = (int64_t*)calloc((size_t)npix, sizeof(int64_t));
  }
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel
  {
    hit_t* hits = NULL;
    int64_t cap = 0;
#pragma omp for schedule(dynamic, 16)
    for (int64_t p = 0; p < npix; ++p) {
      int u = (int)(pix[p] % W), v = (int)(pix[p] / W);
      double d[3];
      cam_dir_raw(cam, u, v, d);
      normalize3(d);
      int64_t nh = collect_hits(&S, o, d, &hits, &cap);
      uint8_t fl = 0;
      for (int64_t h = 1; h < nh; ++h)
        if (hits[h].a - hits[h - 1].a < 1e-9 && hits[h].b > hits[h].a &&
            hits[h - 1].b > hits[h - 1].a)
          fl |= 2;
      /* two passes: pass 0 the plain rule, pass 1 with the first banded
         decision flipped */
      for (int pass = 0; pass < 2; ++pass) {
        double C[3] = {0, 0, 0}, T = 1.0, Dp = 0, Np[3] = {0, 0, 0};
        int flipped = 0;
        int64_t nc = 0;
        for (int64_t h = 0; h < nh; ++h) {
          int stop = T < t_stop;
          if (fabs(T - t_stop) <= band * t_stop) {
            if (pass == 0) fl |= 1;
            if (pass == 1 && !flipped) { stop = !stop; flipped = 1; }
          }
          if (stop) break;
          int64_t i = hits[h].id;
          double x = segment_depth(&S, i, o, d, hits[h].a, hits[h].b, K, act, NULL);
          double alpha = 1.0 - exp(-x);
          double rgb[3], pre[3], Y[16];
          voxel_color(&S, i, o, rgb, pre, Y);
          for (int ch = 0; ch < 3; ++ch) C[ch] += T * alpha * rgb[ch];
          if (pass == 0 && depth)
            Dp += T * segment_local_depth(&S, i, o, d, hits[h].a, hits[h].b, K, act, NULL);
          if (pass == 0 && normal) {
            double n[3];
            voxel_normal(&S, i, n, NULL, NULL);
            for (int ax = 0; ax < 3; ++ax) Np[ax] += T * alpha * n[ax];
          }
          T *= exp(-x);
          if (pass == 0 && seq && nc < max_seq) seq[p * max_seq + nc] = (int32_t)i;
          ++nc;
        }
        double* out = pass == 0 ? rgba : rgba_alt;
        if (out) {
          out[p * 4 + 0] = C[0];
          out[p * 4 + 1] = C[1];
          out[p * 4 + 2] = C[2];
          out[p * 4 + 3] = 1.0 - T;
        }
        if (pass == 0) {
          if (depth) depth[p] = Dp;
          if (normal) for (int ax = 0; ax < 3; ++ax) normal[p * 3 + ax] = Np[ax];
          if (ncomp) ncomp[p] = (int32_t)nc;
          if (nhit) nhit[p] = (int32_t)nh;
          if (seq) for (int64_t q = nc; q < max_seq; ++q) seq[p * max_seq + q] = -1;
          /* adjoint of the plain-rule result (eq. alpha_blend, Supp. A.2   */
          /* gradient of alpha): walk the composited hits back to front     */
          if ((g_rgba || max_weight) && nc > 0) {
            grec_t* R = (grec_t*)malloc((size_t)nc * sizeof(grec_t));
            double* Ti = (double*)malloc((size_t)nc * sizeof(double));
            double* xs = (double*)malloc((size_t)nc * sizeof(double));
            double Tt = 1.0;
            for (int64_t h = 0; h < nc; ++h) {
              Ti[h] = Tt;
              xs[h] = segment_depth(&S, hits[h].id, o, d, hits[h].a, hits[h].b, K, act, NULL);
              R[h].id = hits[h].id;
              R[h].w = Tt * (1.0 - exp(-xs[h]));
              R[h].prio = 0;
              Tt *= exp(-xs[h]);
            }
            double Tfin = Tt;
            const double* g = g_rgba ? g_rgba + p * 4 : NULL;
            double Sfx[3] = {0, 0, 0}; /* colour of the hits behind h, seen from just behind h */
            double SN[3] = {0, 0, 0};  /* the same for the normal */
            double Q = 0;              /* depth of the hits behind h over T_{h+1} */
            const double* gD = (g && g_depth) ? g_depth + p : NULL;
            const double* gN = (g && g_normal) ? g_normal + p * 3 : NULL;
            for (int64_t h = nc - 1; g && h >= 0; --h) {
              int64_t i = hits[h].id;
              double dxdV[8];
              double x = segment_depth(&S, i, o, d, hits[h].a, hits[h].b, K, act, dxdV);
              double alpha = 1.0 - exp(-x);
              double rgb[3];
              R[h].id = i;
              voxel_color(&S, i, o, rgb, R[h].pre, R[h].Y);
              /* dC/dc_h = T_h alpha_h */
              for (int ch = 0; ch < 3; ++ch) R[h].g[8 + ch] = g[ch] * Ti[h] * alpha;
              /* dL/dalpha_h = T_h <g, c_h - S_h> + g_A T_final / (1 - alpha_h);
                 multiplied by dalpha/dx = 1 - alpha_h = exp(-x_h) to avoid the
                 division: dL/dx_h = T_h e^{-x_h} <g, c_h - S_h> + g_A T_final */
              double dot = 0;
              for (int ch = 0; ch < 3; ++ch) dot += g[ch] * (rgb[ch] - Sfx[ch]);
              double dLdx = Ti[h] * exp(-x) * dot + g[3] * Tfin;
              double dLdV_extra[8] = {0, 0, 0, 0, 0, 0, 0, 0};
              double nrm[3] = {0, 0, 0};
              if (gN) {
                /* N = sum T_i alpha_i n_i: as the colour, plus dL/dn_h = T_h alpha_h g_N */
                double dLdn[3];
                for (int ax = 0; ax < 3; ++ax) dLdn[ax] = Ti[h] * alpha * gN[ax];
                voxel_normal(&S, i, nrm, dLdn, dLdV_extra);
                double dn_ = 0;
                for (int ax = 0; ax < 3; ++ax) dn_ += gN[ax] * (nrm[ax] - SN[ax]);
                dLdx += Ti[h] * exp(-x) * dn_;
              }
              double dloc = 0;
              if (gD) {
                /* D = sum T_i d_i: d_h through its own sample alphas, and the
                   hits behind through T: dD/dx_h = -T_{h+1} Q */
                double dddV[8];
                dloc = segment_local_depth(&S, i, o, d, hits[h].a, hits[h].b, K, act, dddV);
                for (int m = 0; m < 8; ++m) dLdV_extra[m] += gD[0] * Ti[h] * dddV[m];
                dLdx += -gD[0] * Ti[h] * exp(-x) * Q;
              }
              for (int m = 0; m < 8; ++m) R[h].g[m] = dLdx * dxdV[m] + dLdV_extra[m];
              /* subdivision priority term (Sec. 3.2.2 eq. priority) from the
                 same dL/dalpha_h, with 1 - alpha_h = exp(-x_h) */
              double dLdalpha = Ti[h] * dot + g[3] * Tfin / exp(-x);
              R[h].prio = fabs(alpha * dLdalpha);
              for (int ch = 0; ch < 3; ++ch) Sfx[ch] = alpha * rgb[ch] + (1.0 - alpha) * Sfx[ch];
              for (int ax = 0; ax < 3; ++ax) SN[ax] = alpha * nrm[ax] + (1.0 - alpha) * SN[ax];
              Q = dloc + exp(-x) * Q;
            }
            free(Ti);
            free(xs);
            recs[p] = R;
            nrec[p] = nc;
          }
        }
        if (!(fl & 1)) {
          if (rgba_alt && pass == 0) {
            for (int q = 0; q < 4; ++q) rgba_alt[p * 4 + q] = rgba[p * 4 + q];
          }
          break;
        }
      }
      if (flags) flags[p] = fl;
    }
    free(hits);
  }
  if (recs) {
    /* deterministic scatter in pixel order */
    if (g_rgba && grad_grid) memset(grad_grid, 0, (size_t)M * sizeof(double));
    if (g_rgba && grad_sh) memset(grad_sh, 0, (size_t)N * nb * 3 * sizeof(double));
    if (max_weight) memset(max_weight, 0, (size_t)N * sizeof(double));
    if (priority) memset(priority, 0, (size_t)N * sizeof(double));
    for (int64_t p = 0; p < npix; ++p) {
      for (int64_t h = 0; h < nrec[p]; ++h) {
        grec_t* r = &recs[p][h];
        if (max_weight && r->w > max_weight[r->id]) max_weight[r->id] = r->w;
        if (priority) priority[r->id] += r->prio;
        if (!g_rgba) continue;
        if (grad_grid)
          for (int m = 0; m < 8; ++m) grad_grid[vox_grid[r->id * 8 + m]] += r->g[m];
        if (grad_sh)
          for (int ch = 0; ch < 3; ++ch) {
            if (!(r->pre[ch] > 0)) continue; /* clamp at 0 passes no gradient */
            for (int j = 0; j < nb; ++j) grad_sh[(r->id * nb + j) * 3 + ch] += r->g[8 + ch] * r->Y[j];
          }
      }
      free(recs[p]);
    }
    free(recs);
    free(nrec);
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Projection to image space (Sec. 3.1.2 "Projection to image space"): the   */
/* 8 corners are projected and the voxel is assigned to every tile that the  */
/* axis-aligned box of the projected points overlaps.  Readings for what the */
/* paper leaves open:                                                        */
/*   - a voxel is culled when all corners lie outside one of the four side  */
/*     planes of the view frustum (image border 0..W, 0..H) or all have     */
/*     camera depth z <= 0;                                                  */
/*   - a voxel with some corner at depth z < z_near is assigned every tile; */
/*   - otherwise pixel (u, v) is covered when its centre (u+0.5, v+0.5) lies */
/*     in the box of the projected corners; tiles are those of the covered  */
/*     pixel range.                                                          */
/* Output per voxel: tile rectangle tx0, tx1, ty0, ty1 (inclusive; empty if  */
/* tx0 > tx1), computed twice: with the projected box shrunk by `band` px    */
/* ("must") and grown by `band` px ("may"); z_near is also banded.           */
/* ------------------------------------------------------------------------ */
void oracle_voxel_tiles(int64_t N, const double* center, const double* size, const double* cam,
                        int tile_w, int tile_h, double z_near, double band, int32_t* rect_must,
                        int32_t* rect_may) {
  int W = (int)cam[0], H = (int)cam[1];
  double fx = cam[2], fy = cam[3], cx = cam[4], cy = cam[5];
  const double* M = cam + 6;
  int ntx = (W + tile_w - 1) / tile_w, nty = (H + tile_h - 1) / tile_h;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < N; ++i) {
    double P[8][3];
    double s = size[i];
    double zmin = INFINITY;
    for (int c = 0; c < 8; ++c) {
      double w[3] = {center[i] + (((c >> 2) & 1) ? 0.5 : -0.5) * s,
                     center[N + i] + (((c >> 1) & 1) ? 0.5 : -0.5) * s,
                     center[2 * N + i] + ((c & 1) ? 0.5 : -0.5) * s};
      for (int r = 0; r < 3; ++r) P[c][r] = M[r * 4 + 0] * w[0] + M[r * 4 + 1] * w[1] + M[r * 4 + 2] * w[2] + M[r * 4 + 3];
      zmin = fmin(zmin, P[c][2]);
    }
    int out[4] = {0, 0, 0, 0};
    for (int c = 0; c < 8; ++c) {
      if (fx * P[c][0] + cx * P[c][2] >= 0) out[0] = 1;
      if (fx * P[c][0] + (cx - W) * P[c][2] <= 0) out[1] = 1;
      if (fy * P[c][1] + cy * P[c][2] >= 0) out[2] = 1;
      if (fy * P[c][1] + (cy - H) * P[c][2] <= 0) out[3] = 1;
    }
    int culled = !(out[0] && out[1] && out[2] && out[3]);
    int behind = 1;
    for (int c = 0; c < 8; ++c) if (P[c][2] > 0) behind = 0;
    for (int which = 0; which < 2; ++which) {
      int32_t* R = (which == 0 ? rect_must : rect_may) + 4 * i;
      double g = which == 0 ? -band : band; /* grow amount */
      R[0] = 1; R[1] = 0; R[2] = 1; R[3] = 0;
      if (culled || behind) continue;
      double zn = which == 0 ? z_near * (1.0 - 1e-3) - 1e-6 : z_near * (1.0 + 1e-3) + 1e-6;
      if (zmin < zn) {
        R[0] = 0; R[1] = ntx - 1; R[2] = 0; R[3] = nty - 1;
        continue;
      }
      double x0 = INFINITY, x1 = -INFINITY, y0 = INFINITY, y1 = -INFINITY;
      for (int c = 0; c < 8; ++c) {
        double x = fx * P[c][0] / P[c][2] + cx;
        double y = fy * P[c][1] / P[c][2] + cy;
        x0 = fmin(x0, x); x1 = fmax(x1, x); y0 = fmin(y0, y); y1 = fmax(y1, y);
      }
      double u0 = ceil(x0 - g - 0.5), u1 = floor(x1 + g - 0.5);
      double v0 = ceil(y0 - g - 0.5), v1 = floor(y1 + g - 0.5);
      u0 = fmax(u0, 0); v0 = fmax(v0, 0); u1 = fmin(u1, W - 1); v1 = fmin(v1, H - 1);
      if (u0 > u1 || v0 > v1) continue;
      R[0] = (int32_t)(u0 / tile_w); R[1] = (int32_t)(u1 / tile_w);
      R[2] = (int32_t)(v0 / tile_h); R[3] = (int32_t)(v1 / tile_h);
    }
  }
}

/* Ray sign bits of every tile (Supp. B.2 "to_rd_signbits"; Supp. B.1: a    */
/* voxel is duplicated per ray-sign pattern that occurs in the tile).  A     */
/* pixel whose direction has a component within rel_band of zero (relative  */
/* to |d|) contributes both signs of that component to `may` and nothing to  */
/* `must`.                                                                   */
void oracle_tile_masks(const double* cam, int tile_w, int tile_h, double rel_band,
                       uint8_t* must, uint8_t* may) {
  int W = (int)cam[0], H = (int)cam[1];
  int ntx = (W + tile_w - 1) / tile_w, nty = (H + tile_h - 1) / tile_h;
  memset(must, 0, (size_t)ntx * nty);
  memset(may, 0, (size_t)ntx * nty);
  for (int v = 0; v < H; ++v)
    for (int u = 0; u < W; ++u) {
      double d[3];
      cam_dir_raw(cam, u, v, d);
      double n = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
      int amb = 0, s = 0;
      for (int ax = 0; ax < 3; ++ax) {
        if (d[ax] < 0) s |= 1 << (2 - ax);
        if (fabs(d[ax]) <= rel_band * n) amb |= 1 << (2 - ax);
      }
      int t = (v / tile_h) * ntx + (u / tile_w);
      if (!amb) must[t] |= (uint8_t)(1u << s);
      for (int f = 0; f < 8; ++f)
        if ((f & ~amb) == 0) may[t] |= (uint8_t)(1u << (s ^ f));
    }
}

/* ------------------------------------------------------------------------ */
/* Anti-aliased downsampling (Sec. 3.1.2 "Anti-aliasing": render ss times    */
/* larger, then downsample with an anti-aliasing filter) and background      */
/* (Supp. implementation details: a background colour fills the remaining   */
/* transmittance).  Reading for the unspecified filter: the separable tent   */
/* of half-width s = n_in / n_out per axis, centred at (i + 1/2) s - 1/2 in  */
/* input pixel coordinates, weights normalised over the in-image taps.       */
/*   out[y][x][c] = sum_{j,k} wy(y,j) wx(x,k) in[j][k][c]                    */
/*   out rgb += (1 - out A) * bg                                             */
/* img layout [h][w][4].                                                     */
/* ------------------------------------------------------------------------ */
static void tent_weights(int n_in, int n_out, int i, int* j0, int* j1, double* w) {
  double s = (double)n_in / (double)n_out;
  double c = (i + 0.5) * s - 0.5;
  int lo = (int)floor(c - s), hi = (int)ceil(c + s);
  if (lo < 0) lo = 0;
  if (hi > n_in - 1) hi = n_in - 1;
  double tot = 0;
  for (int j = lo; j <= hi; ++j) {
    double t = 1.0 - fabs((double)j - c) / s;
    w[j - lo] = t > 0 ? t : 0;
    tot += w[j - lo];
  }
  for (int j = lo; j <= hi; ++j) w[j - lo] /= tot;
  *j0 = lo;
  *j1 = hi;
}

void oracle_downsample(const double* in, int w_in, int h_in, double* out, int w_out, int h_out,
                       const double* bg) {
  double* wx = (double*)malloc((size_t)(2 * w_in + 4) * sizeof(double));
  double* wy = (double*)malloc((size_t)(2 * h_in + 4) * sizeof(double));
  for (int y = 0; y < h_out; ++y) {
    int y0, y1;
    tent_weights(h_in, h_out, y, &y0, &y1, wy);
    for (int x = 0; x < w_out; ++x) {
      int x0, x1;
      tent_weights(w_in, w_out, x, &x0, &x1, wx);
      double acc[4] = {0, 0, 0, 0};
      for (int j = y0; j <= y1; ++j)
        for (int k = x0; k <= x1; ++k)
          for (int c = 0; c < 4; ++c)
            acc[c] += wy[j - y0] * wx[k - x0] * in[((size_t)j * w_in + k) * 4 + c];
      if (bg)
        for (int c = 0; c < 3; ++c) acc[c] += (1.0 - acc[3]) * bg[c];
      for (int c = 0; c < 4; ++c) out[((size_t)y * w_out + x) * 4 + c] = acc[c];
    }
  }
  free(wx);
  free(wy);
}

/* adjoint of oracle_downsample: grad_in = D^T grad_out for the linear map D  */
/* above (the background term makes out rgb depend on out A: its gradient   */
/* adds -<g_rgb, bg> to the alpha channel before the transpose)             */
void oracle_downsample_adjoint(const double* gout, int w_out, int h_out, double* gin, int w_in,
                               int h_in, const double* bg) {
  double* wx = (double*)malloc((size_t)(2 * w_in + 4) * sizeof(double));
  double* wy = (double*)malloc((size_t)(2 * h_in + 4) * sizeof(double));
  memset(gin, 0, (size_t)w_in * h_in * 4 * sizeof(double));
  for (int y = 0; y < h_out; ++y) {
    int y0, y1;
    tent_weights(h_in, h_out, y, &y0, &y1, wy);
    for (int x = 0; x < w_out; ++x) {
      int x0, x1;
      tent_weights(w_in, w_out, x, &x0, &x1, wx);
      const double* g = gout + ((size_t)y * w_out + x) * 4;
      double ge[4] = {g[0], g[1], g[2], g[3]};
      if (bg) ge[3] -= g[0] * bg[0] + g[1] * bg[1] + g[2] * bg[2];
      for (int j = y0; j <= y1; ++j)
        for (int k = x0; k <= x1; ++k)
          for (int c = 0; c < 4; ++c)
            gin[((size_t)j * w_in + k) * 4 + c] += wy[j - y0] * wx[k - x0] * ge[c];
    }
  }
  free(wx);
  free(wy);
}
