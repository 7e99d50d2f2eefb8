// Host-only harness of the C ABI's argument checks and workspace layout,
// built with AddressSanitizer and UndefinedBehaviorSanitizer on the host
// code by tests/test_sanitizers.py.  No call here reaches a kernel launch:
// every one returns from its host-side checks (the pointers are never
// dereferenced), so it runs without a GPU.
#include <stdio.h>
#include <string.h>

#include <initializer_list>

#include "svraster.h"

static int fails = 0;
#define EXPECT(cond)                                                   \
  do {                                                                 \
    if (!(cond)) {                                                     \
      fprintf(stderr, "line %d: %s (%s)\n", __LINE__, #cond, svr_last_error()); \
      ++fails;                                                         \
    }                                                                  \
  } while (0)

int main() {
  void* fake = reinterpret_cast<void*>(0x10000);
  svr_scene sc;
  memset(&sc, 0, sizeof(sc));
  sc.n_voxels = 1000;
  sc.n_grid = 2000;
  sc.center = static_cast<const float*>(fake);
  sc.size = static_cast<const float*>(fake);
  sc.octpath = static_cast<const uint64_t*>(fake);
  sc.vox_grid = static_cast<const int32_t*>(fake);
  sc.grid_raw = static_cast<const float*>(fake);
  sc.sh = static_cast<const float*>(fake);
  sc.sh_degree = 3;
  sc.max_level = 12;
  svr_camera cams[3];
  memset(cams, 0, sizeof(cams));
  for (int i = 0; i < 3; ++i) {
    cams[i].width = 64 + 37 * i;
    cams[i].height = 48 + 5 * i;
    cams[i].fx = cams[i].fy = 50.f;
    cams[i].cx = cams[i].width / 2.f;
    cams[i].cy = cams[i].height / 2.f;
    const float w2c[12] = {1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 3};
    memcpy(cams[i].w2c, w2c, sizeof(w2c));
  }
  svr_opts o;
  memset(&o, 0, sizeof(o));
  o.K = 2;
  o.t_stop = 1e-4f;
  o.entry_capacity = 4096;
  for (int tile : {0, 8, 16, 32}) {
    o.tile = tile;
    for (int n = 1; n <= 3; ++n) {
      const size_t b = svr_workspace_bytes(&sc, cams, n, &o);
      EXPECT(b > 0);
      size_t parts[SVR_WS_PARTS];
      EXPECT(svr_workspace_parts(&sc, cams, n, &o, parts, SVR_WS_PARTS) == SVR_OK);
      size_t tot = 0;
      for (int k = 0; k < SVR_WS_PARTS; ++k) tot += parts[k];
      EXPECT(tot <= b);
      // a workspace one byte short is refused before anything runs
      EXPECT(svr_preprocess(&sc, cams, n, &o, fake, b - 1, nullptr, nullptr) == SVR_E_WORKSPACE);
    }
  }
  o.tile = 8;
  const size_t ws = svr_workspace_bytes(&sc, cams, 1, &o);
  // bad options and scenes
  svr_opts bad = o;
  bad.K = 0;
  EXPECT(svr_preprocess(&sc, cams, 1, &bad, fake, ws, nullptr, nullptr) == SVR_E_INVALID);
  bad = o;
  bad.tile = 12;
  EXPECT(svr_workspace_bytes(&sc, cams, 1, &bad) == 0);
  bad = o;
  bad.entry_capacity = (int64_t)1 << 30;
  EXPECT(svr_sort(&sc, cams, 1, &bad, fake, ws, -1, nullptr) == SVR_E_INVALID);
  svr_scene bs = sc;
  bs.sh_degree = 4;
  EXPECT(svr_render_fwd(&bs, cams, 1, &o, fake, ws, static_cast<float*>(fake), nullptr, nullptr) ==
         SVR_E_INVALID);
  bs = sc;
  bs.center = nullptr;
  EXPECT(svr_render_bwd(&bs, cams, 1, &o, fake, ws, static_cast<const float*>(fake), nullptr,
                        nullptr, nullptr, nullptr) == SVR_E_INVALID);
  EXPECT(svr_render_fwd(&sc, cams, 1, &o, fake, ws, nullptr, nullptr, nullptr) == SVR_E_INVALID);
  EXPECT(svr_preprocess(&sc, nullptr, 1, &o, fake, ws, nullptr, nullptr) == SVR_E_INVALID);
  EXPECT(svr_preprocess(&sc, cams, 0, &o, fake, ws, nullptr, nullptr) == SVR_E_INVALID);
  EXPECT(svr_preprocess(&sc, cams, SVR_MAX_CAMERAS + 1, &o, fake, ws, nullptr, nullptr) ==
         SVR_E_INVALID);
  svr_camera bc = cams[0];
  bc.fx = -1.f;
  EXPECT(svr_preprocess(&sc, &bc, 1, &o, fake, ws, nullptr, nullptr) == SVR_E_INVALID);
  bc = cams[0];
  bc.width = 20000;
  EXPECT(svr_workspace_bytes(&sc, &bc, 1, &o) == 0);
  // stand-alone sorts and helpers
  EXPECT(svr_radix_sort_scratch_bytes(-1, 8) == 0);
  EXPECT(svr_radix_sort_pairs(nullptr, nullptr, nullptr, nullptr, 10, 8, nullptr, 0, nullptr) ==
         SVR_E_INVALID);
  EXPECT(svr_radix_sort_pairs_static(static_cast<uint64_t*>(fake), static_cast<uint32_t*>(fake),
                                     (int64_t)SVR_STATIC_SORT_MAX + 1, 32, nullptr) == SVR_E_INVALID);
  EXPECT(svr_radix_sort_pairs_static(nullptr, nullptr, 5, 65, nullptr) == SVR_E_INVALID);
  EXPECT(svr_atomic_probe(nullptr, nullptr, 10, 10, 1, nullptr) == SVR_E_INVALID);
  EXPECT(svr_atomic_probe(static_cast<float*>(fake), static_cast<float*>(fake), 0, 10, 1,
                          nullptr) == SVR_E_INVALID);
  EXPECT(svr_order_rank_scratch_bytes(-1, 12) == 0);
  EXPECT(svr_grid_adjacency_scratch_bytes(-1, 5) == 0);
  for (int st = 1; st >= -6; --st) EXPECT(svr_status_string(st) != nullptr);
  if (fails) return 1;
  printf("abi harness ok\n");
  return 0;
}
