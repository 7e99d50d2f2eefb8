/* Host-only harness: every function of the FP64 oracle on a small scene,
 * built with AddressSanitizer and UndefinedBehaviorSanitizer by
 * tests/test_sanitizers.py.  Exits 0 when every call completes; the
 * sanitizers abort on the first finding.  The scene: the 8 level-1 voxels
 * of the unit cube with the shared 3x3x3 corner grid, random densities and
 * degree-3 SH coefficients, seen by a 21x13 camera (ragged 8x8 tiles). */
#include <stdio.h>
#include <stdlib.h>

#include "../../oracle/svr_oracle.c"

static double rnd(unsigned* s) {
  *s = *s * 1664525u + 1013904223u;
  return (double)(*s >> 8) / 16777216.0;
}

int main(void) {
  enum { N = 8, M = 27, D = 3, NB = 16, W = 21, H = 13 };
  unsigned seed = 12345u;
  double center[3 * N], size[N], raw[M], sh[N * NB * 3];
  int32_t vg[N * 8];
  uint64_t path[N];
  for (int v = 0; v < N; ++v) {
    int i = (v >> 2) & 1, j = (v >> 1) & 1, k = v & 1;
    center[v] = 0.25 + 0.5 * i;
    center[N + v] = 0.25 + 0.5 * j;
    center[2 * N + v] = 0.25 + 0.5 * k;
    size[v] = 0.5;
    path[v] = oracle_to_octpath(i, j, k, 1);
    for (int c = 0; c < 8; ++c) {
      int gi = i + ((c >> 2) & 1), gj = j + ((c >> 1) & 1), gk = k + (c & 1);
      vg[8 * v + c] = (gi * 3 + gj) * 3 + gk;
    }
  }
  for (int m = 0; m < M; ++m) raw[m] = 4.0 * rnd(&seed) - 1.0;
  for (int q = 0; q < N * NB * 3; ++q) sh[q] = rnd(&seed) - 0.5;
  /* camera at (1.7, 1.3, 1.9) looking at the cube centre: R rows right,
   * down, forward */
  double eye[3] = {1.7, 1.3, 1.9}, fwd[3], up[3] = {0, 0, 1}, right[3], down[3];
  double nf = 0;
  for (int c = 0; c < 3; ++c) { fwd[c] = 0.5 - eye[c]; nf += fwd[c] * fwd[c]; }
  nf = sqrt(nf);
  for (int c = 0; c < 3; ++c) fwd[c] /= nf;
  right[0] = fwd[1] * up[2] - fwd[2] * up[1];
  right[1] = fwd[2] * up[0] - fwd[0] * up[2];
  right[2] = fwd[0] * up[1] - fwd[1] * up[0];
  double nr = sqrt(right[0] * right[0] + right[1] * right[1] + right[2] * right[2]);
  for (int c = 0; c < 3; ++c) right[c] /= nr;
  down[0] = fwd[1] * right[2] - fwd[2] * right[1];
  down[1] = fwd[2] * right[0] - fwd[0] * right[2];
  down[2] = fwd[0] * right[1] - fwd[1] * right[0];
  double cam[18] = {W, H, 18.0, 18.0, 0.5 * W, 0.5 * H};
  const double* rows[3] = {right, down, fwd};
  for (int r = 0; r < 3; ++r) {
    double t = 0;
    for (int c = 0; c < 3; ++c) { cam[6 + 4 * r + c] = rows[r][c]; t -= rows[r][c] * eye[c]; }
    cam[6 + 4 * r + 3] = t;
  }
  const int64_t P = W * H;
  int64_t* pix = malloc(P * sizeof(int64_t));
  for (int64_t p = 0; p < P; ++p) pix[p] = p;
  double* rgba = calloc(P * 4, sizeof(double));
  double* alt = calloc(P * 4, sizeof(double));
  uint8_t* flags = calloc(P, 1);
  int32_t* ncomp = calloc(P, sizeof(int32_t));
  int32_t* nhit = calloc(P, sizeof(int32_t));
  int32_t* seq = calloc(P * 8, sizeof(int32_t));
  double* g = malloc(P * 4 * sizeof(double));
  double* gd = malloc(P * sizeof(double));
  double* gn = malloc(P * 3 * sizeof(double));
  for (int64_t q = 0; q < P * 4; ++q) g[q] = rnd(&seed) - 0.5;
  for (int64_t q = 0; q < P; ++q) gd[q] = rnd(&seed) - 0.5;
  for (int64_t q = 0; q < P * 3; ++q) gn[q] = rnd(&seed) - 0.5;
  double* gg = calloc(M, sizeof(double));
  double* gs = calloc(N * NB * 3, sizeof(double));
  double* mw = calloc(N, sizeof(double));
  double* pr = calloc(N, sizeof(double));
  double* dep = calloc(P, sizeof(double));
  double* nrm = calloc(P * 3, sizeof(double));
  for (int K = 1; K <= 3; ++K)
    for (int act = 0; act < 2; ++act)
      oracle_render(N, center, size, vg, raw, M, sh, D, cam, K, 1e-4, act, 1e-3, P, pix, rgba, alt,
                    flags, ncomp, nhit, seq, 8, g, gg, gs, mw, pr, dep, nrm, gd, gn, 2);
  int32_t must[N * 4], may[N * 4];
  oracle_voxel_tiles(N, center, size, cam, 8, 8, 1e-4, 0.02, must, may);
  const int ntiles = ((W + 7) / 8) * ((H + 7) / 8);
  uint8_t m_must[16], m_may[16];
  oracle_tile_masks(cam, 8, 8, 1e-6, m_must, m_may);
  int64_t tile[8 * N], vid[8 * N];
  uint8_t sg[8 * N];
  for (int e = 0; e < 8 * N; ++e) { tile[e] = e % ntiles; vid[e] = e / 8; sg[e] = (uint8_t)(e % 8); }
  uint64_t kp[8 * N], kc[8 * N];
  uint32_t val[8 * N];
  oracle_keys(8 * N, tile, vid, sg, path, 1, kp, kc, val);
  int64_t ijk[3];
  for (int v = 0; v < N; ++v) oracle_to_voxel_index(path[v], 1, ijk);
  for (int s = 0; s < 8; ++s)
    for (int t = 0; t < 8; ++t) (void)oracle_child_rank(s, t);
  double Y[16], dir[3] = {0.3, -0.4, 0.5};
  for (int d = 0; d <= 3; ++d) oracle_sh_basis(d, dir, Y);
  double* small = calloc((size_t)(W - 5) * (H - 3) * 4, sizeof(double));
  double bg[3] = {0.2, 0.3, 0.4};
  oracle_downsample(rgba, W, H, small, W - 5, H - 3, bg);
  oracle_downsample_adjoint(small, W - 5, H - 3, rgba, W, H, bg);
  double total = 0;
  for (int m = 0; m < M; ++m) total += gg[m];
  printf("oracle harness ok (%d x %d px, sum grad_grid %.6g)\n", W, H, total);
  free(pix); free(rgba); free(alt); free(flags); free(ncomp); free(nhit); free(seq);
  free(g); free(gd); free(gn); free(gg); free(gs); free(mw); free(pr); free(dep); free(nrm);
  free(small);
  return 0;
}
