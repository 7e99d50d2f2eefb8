"""GPU parity: the HIP path, called through the C ABI, against the FP64 oracle
(bars in parity_helpers: sorted lists bit-exact, RGBA within 1e-4, gradients
within 1e-3 relative)."""
import math

import numpy as np
import pytest

import oracle
from paper_2412_04459_amd import scenes as S
from parity_helpers import (GRAD_FLOOR, GRAD_REL, RGBA_TOL, check_grad as _check_grad,
                            check_rgba as _check_rgba, check_sorted_list,
                            cpu_order_ranks as _cpu_order_ranks, say as _say)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _gpu_frame(torch, scene, cams, K, t_stop=1e-4, act=0, grad=None, sync=True, tile=16,
               ranks=True):
    from paper_2412_04459_amd.render import DeviceScene, Rasterizer
    ds = DeviceScene(scene, order_ranks=ranks)
    rast = Rasterizer(ds, cams, K=K, t_stop=t_stop, activation=act, sync_count=sync, tile=tile)
    rgba = rast.forward()
    out = {"rast": rast, "rgba": rgba.cpu().numpy().astype(np.float64)}
    if grad is not None:
        gg, gs = rast.backward(torch.from_numpy(np.ascontiguousarray(grad, np.float32)).cuda())
        out["grad_grid"] = gg.cpu().numpy().astype(np.float64)
        out["grad_sh"] = gs.cpu().numpy().astype(np.float64)
    torch.cuda.synchronize()
    return out


# ---------------------------------------------------------------------------
# radix sort (bit-exact against a stable sort of the same list)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n,bits", [(1, 8), (100, 8), (2047, 12), (2048, 30), (2049, 30),
                                    (4095, 20), (4096, 52), (4097, 52),
                                    (100_003, 36), (1_500_000, 52), (300_000, 64)])
def test_radix_sort_matches_stable_sort(torch_dev, n, bits):
    torch = torch_dev
    from paper_2412_04459_amd.render import radix_sort_pairs
    _say("radix sort n=%d bits=%d" % (n, bits))
    rng = np.random.default_rng(n + bits)
    keys = rng.integers(0, 2 ** 63, size=n, dtype=np.int64).view(np.uint64)
    keys[: n // 3] = keys[: n // 3] % np.uint64(97)  # many duplicates
    if bits < 64:
        # keys above the sorted bits are left as they are; only [0, bits) counts
        pass
    vals = np.arange(n, dtype=np.int32)
    kt = torch.from_numpy(keys.view(np.int64).copy()).cuda()
    vt = torch.from_numpy(vals.copy()).cuda()
    radix_sort_pairs(kt, vt, bits)
    torch.cuda.synchronize()
    mask = np.uint64((1 << bits) - 1) if bits < 64 else np.uint64(0xFFFFFFFFFFFFFFFF)
    order = np.argsort(keys & mask, kind="stable")
    assert np.array_equal(vt.cpu().numpy(), vals[order])
    assert np.array_equal(kt.cpu().numpy().view(np.uint64), keys[order])


# ---------------------------------------------------------------------------
# duplicated, sorted (key, value) list
# ---------------------------------------------------------------------------
def _key_cases():
    return [("shell", lambda: (S.sphere_shell_scene(), [S.sphere_shell_camera()])),
            ("shell_ragged", lambda: (S.sphere_shell_scene(), [S.look_at(77, 51, 60.0, [1.5, -1.2, 1.0],
                                                                  target=(0.3, 0.3, 0.3))])),
            ("spheres_plane", lambda: (S.spheres_plane_scene(), [S.spheres_plane_camera()])),
            ("tiny_multisign", lambda: (S.tiny_random_scene(4, max_level=4),
                                        [S.look_at(90, 70, 100.0, [0.5, 0.45, 0.55],
                                                   target=(0.9, 0.8, 0.7))])),
            # a single 16x16 tile over a dense 32^3 block of voxels: ~16k
            # entries in one range, past the in-LDS sort of a tile's range
            ("one_tile", lambda: (_dense_cube(5), [S.look_at(16, 16, 20.0, [1.9, 1.7, 1.5],
                                                             target=(0.5, 0.5, 0.5))]))]


def _dense_cube(level):
    """Every voxel of level `level` in the unit cube (zero densities)."""
    n = 1 << level
    g = np.stack(np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij"), -1).reshape(-1, 3)
    return S.scene_from_voxels((0.5, 0.5, 0.5), 1.0, level, g, np.full(len(g), level))




@pytest.mark.parametrize("name,ranks", [(c[0], True) for c in _key_cases()] + [("shell", False),
                                                                             ("tiny_multisign", False),
                                                                             ("one_tile", False)])
def test_sorted_entries_bit_exact(torch_dev, name, ranks):
    torch = torch_dev
    make = dict(_key_cases())[name]
    scene, cams = make()
    _say("sorted entries: %s N=%d %dx%d ranks=%d" % (name, scene.n_voxels, cams[0].W, cams[0].H,
                                                     ranks))
    out = _gpu_frame(torch, scene, cams, K=1, ranks=ranks)
    rast = out["rast"]
    E = rast.n_entries
    keys, vals = rast.sorted_entries(E)
    assert rast.check_overflow() == E
    if name == "one_tile":
        assert E > 2048  # the range is sorted by the radix fallback
    check_sorted_list(scene, cams[0], keys.cpu().numpy().view(np.uint64),
                       vals.cpu().numpy().view(np.uint32), ranks)


def test_second_sort_after_one_preprocess(torch_dev):
    """The per-tile counts of the counting sort start at zero for a second
    sort of the same emitted list (the tile-order pass clears them), so the
    list and the header check come out unchanged."""
    torch = torch_dev
    from paper_2412_04459_amd.render import DeviceScene, Rasterizer
    scene, cams = S.spheres_plane_scene(), [S.spheres_plane_camera()]
    _say("second sort: spheres_plane N=%d" % scene.n_voxels)
    rast = Rasterizer(DeviceScene(scene), cams, K=1, sync_count=True, tile=8)
    rast.preprocess()
    rast.sort()
    E = rast.n_entries
    k1, v1 = [t.cpu().numpy() for t in rast.sorted_entries(E)]
    assert rast.check_overflow() == E
    rast.sort()
    k2, v2 = [t.cpu().numpy() for t in rast.sorted_entries(E)]
    assert rast.check_overflow() == E
    assert np.array_equal(k1, k2) and np.array_equal(v1, v2)
    check_sorted_list(scene, cams[0], k2.view(np.uint64), v2.view(np.uint32), True, tile=8)


def test_counting_sort_at_its_tile_limit(torch_dev):
    """A 1920x1080 view at 8x8 tiles has 32,400 tiles, just under the counting
    sort's 32,768 (its per-tile histogram then takes ~127 KB of LDS): the
    sorted list is still the oracle's."""
    torch = torch_dev
    from paper_2412_04459_amd.render import DeviceScene, Rasterizer
    scene = S.spheres_plane_scene()
    cam = S.look_at(1920, 1080, 60.0, [1.5, 1.2, 1.0])
    assert ((cam.W + 7) // 8) * ((cam.H + 7) // 8) == 32400
    _say("counting sort at 32400 tiles: N=%d" % scene.n_voxels)
    rast = Rasterizer(DeviceScene(scene), [cam], K=1, sync_count=True, tile=8)
    rast.preprocess()
    rast.sort()
    E = rast.n_entries
    keys, vals = rast.sorted_entries(E)
    assert rast.check_overflow() == E
    check_sorted_list(scene, cam, keys.cpu().numpy().view(np.uint64),
                      vals.cpu().numpy().view(np.uint32), True, tile=8)


@pytest.mark.parametrize("graph", [False, True])
def test_view_without_entries(torch_dev, graph):
    """A camera facing away from the scene: every voxel is culled, E = 0, the
    counting sort sees an empty list, and the image and the gradients are
    zero, as the oracle's."""
    torch = torch_dev
    from paper_2412_04459_amd.render import DeviceScene, Rasterizer
    scene = S.sphere_shell_scene()
    cam = S.look_at(48, 40, 60.0, [3.0, 0.0, 0.0], target=(6.0, 0.0, 0.0))
    _say("view without entries: graph=%d" % graph)
    ref = oracle.render(scene, cam, K=1, grad_rgba=np.ones((cam.W * cam.H, 4)))
    assert np.all(ref["rgba"] == 0.0)
    ds = DeviceScene(scene)
    rast = Rasterizer(ds, [cam], K=1, sync_count=not graph, tile=8)
    g = torch.ones((cam.W * cam.H, 4), dtype=torch.float32, device="cuda")
    if graph:
        # outputs start as garbage: the replays must overwrite them
        rgba = torch.full((cam.W * cam.H, 4), -1.0, dtype=torch.float32, device="cuda")
        gg = torch.full((ds.n_grid,), 7.0, dtype=torch.float32, device="cuda")
        gs = torch.full_like(ds.sh, 7.0)
        stream = torch.cuda.Stream()
        assert rast.capture_views([cam], rgba, g, gg, gs, stream) == 1
        for _ in range(2):
            rast.replay_view(0, stream)
    else:
        rgba = rast.forward()
        gg, gs = rast.backward(g)
    torch.cuda.synchronize()
    assert rast.check_overflow() == 0
    assert float(rgba.abs().max()) == 0.0
    assert float(gg.abs().max()) == 0.0 and float(gs.abs().max()) == 0.0


# ---------------------------------------------------------------------------
# forward RGBA
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("case,K,act", [("shell", 1, 0), ("shell_opaque", 1, 0), ("shell_opaque", 3, 1),
                                        ("ragged_opaque", 2, 0), ("tiny", 4, 0)])
def test_render_fwd_matches_oracle(torch_dev, case, K, act):
    torch = torch_dev
    if case == "shell":
        scene, cams = S.sphere_shell_scene(), [S.sphere_shell_camera()]
    elif case == "shell_opaque":
        scene, cams = S.sphere_shell_scene(opaque=True), [S.sphere_shell_camera()]
    elif case == "ragged_opaque":
        scene = S.sphere_shell_scene(opaque=True)
        cams = [S.look_at(77, 51, 60.0, [1.5, -1.2, 1.0], target=(0.3, 0.3, 0.3))]
    else:
        scene = S.tiny_random_scene(9, max_level=4, sh_degree=3)
        cams = [S.look_at(90, 70, 80.0, [1.7, 1.4, 1.2], target=(0.5, 0.5, 0.5))]
    _say("render fwd %s K=%d act=%d" % (case, K, act))
    out = _gpu_frame(torch, scene, cams, K=K, act=act)
    ref = oracle.render(scene, cams[0], K=K, activation=act)
    err = _check_rgba(out["rgba"], ref)
    assert ref["rgba"][:, 3].max() > 0.1
    _say("  max err %.3g" % err)


def test_render_fwd_spheres_plane_sampled(torch_dev):
    torch = torch_dev
    scene, cams = S.spheres_plane_scene(), [S.spheres_plane_camera()]
    _say("render fwd spheres+plane sampled")
    out = _gpu_frame(torch, scene, cams, K=1)
    rng = np.random.default_rng(11)
    # sample among pixels with hits and some empty ones
    hit_px = np.nonzero(out["rgba"][:, 3] > 0)[0]
    px = np.concatenate([rng.choice(hit_px, 1500, replace=False),
                         rng.choice(cams[0].W * cams[0].H, 300, replace=False)])
    ref = oracle.render(scene, cams[0], K=1, pixels=px)
    _check_rgba(out["rgba"], ref, pixels=px)


# ---------------------------------------------------------------------------
# gradients
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("case,K,act", [("shell", 1, 0), ("shell_opaque", 2, 0), ("tiny", 3, 1),
                                        ("tiny_opaque", 2, 0)])
def test_render_bwd_matches_oracle(torch_dev, case, K, act):
    torch = torch_dev
    import dataclasses
    if case.startswith("shell"):
        scene, cams = S.sphere_shell_scene(opaque=case.endswith("opaque")), [S.sphere_shell_camera()]
    else:
        scene = S.tiny_random_scene(9, max_level=4, sh_degree=3)
        if case.endswith("opaque"):
            scene = dataclasses.replace(scene, grid_raw=(scene.grid_raw * 8).astype(np.float32))
        cams = [S.look_at(90, 70, 80.0, [1.7, 1.4, 1.2], target=(0.5, 0.5, 0.5))]
    _say("render bwd %s K=%d act=%d" % (case, K, act))
    P = cams[0].W * cams[0].H
    g = S.upstream_grads(P, 5)
    ref0 = oracle.render(scene, cams[0], K=K, activation=act)
    g[ref0["flags"] != 0] = 0.0
    ref = oracle.render(scene, cams[0], K=K, activation=act, grad_rgba=g.astype(np.float64))
    out = _gpu_frame(torch, scene, cams, K=K, act=act, grad=g)
    _check_rgba(out["rgba"], ref0)
    _check_grad(out["grad_grid"], ref["grad_grid"], "grad_grid")
    _check_grad(out["grad_sh"], ref["grad_sh"], "grad_sh")


@pytest.mark.parametrize("tile,K,act", [(8, 2, 0), (32, 1, 1), (16, 3, 0)])
def test_render_bwd_split_heavy_tiles(torch_dev, tile, K, act):
    """Tiles with more than 256 entries run their backward as 256-entry chunks,
    one workgroup each, started from the forward's checkpoints.  The opaque
    shell has tiles of several chunks with early termination inside them; the
    gradients must match the oracle as for unsplit tiles."""
    torch = torch_dev
    scene, cams = S.sphere_shell_scene(opaque=True), [S.sphere_shell_camera()]
    _say("render bwd, split tiles, tile %d K=%d act=%d" % (tile, K, act))
    P = cams[0].W * cams[0].H
    g = S.upstream_grads(P, 6)
    ref0 = oracle.render(scene, cams[0], K=K, activation=act)
    g[ref0["flags"] != 0] = 0.0
    ref = oracle.render(scene, cams[0], K=K, activation=act, grad_rgba=g.astype(np.float64))
    out = _gpu_frame(torch, scene, cams, K=K, act=act, grad=g, tile=tile)
    rast = out["rast"]
    keys, _ = rast.sorted_entries(rast.n_entries)
    tiles = keys.cpu().numpy().view(np.uint64) >> np.uint64(int(8 * scene.n_voxels - 1).bit_length())
    per_tile = np.bincount(tiles.astype(np.int64))
    assert per_tile.max() > 2 * 256, "no tile of three or more chunks"
    _check_rgba(out["rgba"], ref0)
    _check_grad(out["grad_grid"], ref["grad_grid"], "grad_grid")
    _check_grad(out["grad_sh"], ref["grad_sh"], "grad_sh")


def test_render_bwd_spheres_plane_sampled(torch_dev):
    torch = torch_dev
    scene, cams = S.spheres_plane_scene(), [S.spheres_plane_camera()]
    _say("render bwd spheres+plane sampled")
    P = cams[0].W * cams[0].H
    rng = np.random.default_rng(12)
    px = rng.choice(P, 3000, replace=False)
    g_full = np.zeros((P, 4), np.float32)
    g_full[px] = S.upstream_grads(P, 1)[px]
    ref0 = oracle.render(scene, cams[0], K=1, pixels=px)
    g_full[px[ref0["flags"] != 0]] = 0.0
    ref = oracle.render(scene, cams[0], K=1, pixels=px, grad_rgba=g_full[px].astype(np.float64))
    out = _gpu_frame(torch, scene, cams, K=1, grad=g_full)
    _check_grad(out["grad_grid"], ref["grad_grid"], "grad_grid")
    _check_grad(out["grad_sh"], ref["grad_sh"], "grad_sh")


def test_autograd_function_matches_direct_backward(torch_dev):
    torch = torch_dev
    from paper_2412_04459_amd.render import DeviceScene, Rasterizer, render
    scene, cams = S.sphere_shell_scene(opaque=True), [S.sphere_shell_camera()]
    ds = DeviceScene(scene)
    rast = Rasterizer(ds, cams, K=2)
    grid = ds.grid_raw.clone().requires_grad_(True)
    sh = ds.sh.clone().requires_grad_(True)
    rgba = render(rast, grid, sh)
    g = torch.from_numpy(S.upstream_grads(rgba.shape[0], 7)).cuda()
    (rgba * g).sum().backward()
    gg, gs = rast.backward(g)
    torch.cuda.synchronize()
    assert torch.allclose(grid.grad, gg, rtol=1e-5, atol=1e-7)
    assert torch.allclose(sh.grad, gs, rtol=1e-5, atol=1e-7)


# ---------------------------------------------------------------------------
# the benchmark workload (about 1.07M voxels, 1297x840, K = 2): sampled pixels
# against the oracle, both eagerly with the entry count read back and in the
# configuration the benchmark times (8x8 tiles, no host synchronisation, the
# sort sized to the capacity, the whole frame replayed from a captured hipGraph)
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def bench_scene(torch_dev):
    from paper_2412_04459_amd.render import zcurve_relabel
    # stored in octree-path order, as the benchmark stores it
    scene, _ = zcurve_relabel(S.spheres_background_scene())
    cams = S.orbit_cameras_1297x840()[:1]
    return scene, cams


@pytest.fixture(scope="module")
def bench_device_scene(torch_dev, bench_scene):
    from paper_2412_04459_amd.render import DeviceScene
    return DeviceScene(bench_scene[0])


@pytest.fixture(scope="module")
def bench_rank_table(bench_scene):
    return _cpu_order_ranks(bench_scene[0])


def _bench_frame(torch, ds, cam, mode, tile, grad):
    """One fwd+bwd frame of `cam`.  mode 'eager': entry count read back, sort
    sized to it, eager launches.  mode 'graph': capacity from a counted probe
    (as the benchmark sizes it), no host synchronisation, the frame captured
    as one hipGraph and replayed twice (outputs are overwritten per replay).
    Returns (rasterizer, rgba, grad_grid, grad_sh, entries)."""
    from paper_2412_04459_amd.render import Rasterizer
    g = torch.from_numpy(np.ascontiguousarray(grad, np.float32)).cuda()
    if mode == "eager":
        r = Rasterizer(ds, [cam], K=2, sync_count=True, tile=tile)
        rgba = r.forward()
        gg, gs = r.backward(g)
        torch.cuda.synchronize()
        return r, rgba, gg, gs, r.n_entries
    probe = Rasterizer(ds, [cam], K=2, sync_count=True, tile=tile)
    probe.preprocess()
    cap = int(probe.n_entries * 1.1) + 4096
    del probe
    r = Rasterizer(ds, [cam], K=2, capacity=cap, sync_count=False, tile=tile)
    P = cam.W * cam.H
    rgba = torch.full((P, 4), -1.0, dtype=torch.float32, device="cuda")
    gg = torch.full((ds.n_grid,), 7.0, dtype=torch.float32, device="cuda")
    gs = torch.full_like(ds.sh, 7.0)
    stream = torch.cuda.Stream()
    assert r.capture_views([cam], rgba, g, gg, gs, stream) == 1
    for _ in range(2):
        r.replay_view(0, stream)
    torch.cuda.synchronize()
    E = r.check_overflow()
    assert 0 < E <= cap
    return r, rgba, gg, gs, E


@pytest.fixture(scope="module")
def bench_sample(torch_dev, bench_scene, bench_device_scene):
    """A seeded sample of 700 pixels with hits and 100 random pixels of the
    benchmark view, the oracle's rgba there, and the oracle's gradients for an
    upstream gradient that is N(0, 1) on the sample (zero on flagged pixels)
    and zero elsewhere."""
    torch = torch_dev
    scene, cams = bench_scene
    cam = cams[0]
    P = cam.W * cam.H
    _, rgba, _, _, _ = _bench_frame(torch, bench_device_scene, cam, "eager", 16, np.zeros((P, 4)))
    hit_px = np.nonzero(rgba[:, 3].cpu().numpy() > 0)[0]
    rng = np.random.default_rng(13)
    px = np.unique(np.concatenate([rng.choice(hit_px, 700, replace=False),
                                   rng.choice(P, 100, replace=False)]))
    ref0 = oracle.render(scene, cam, K=2, pixels=px)
    g = np.zeros((P, 4), np.float32)
    g[px] = S.upstream_grads(P, 2)[px]
    g[px[ref0["flags"] != 0]] = 0.0
    ref = oracle.render(scene, cam, K=2, pixels=px, grad_rgba=g[px].astype(np.float64))
    return px, g, ref0, ref


@pytest.mark.parametrize("mode,tile", [("eager", 16), ("eager", 8), ("graph", 8), ("graph", 16)])
def test_bench_scene_sampled_parity(torch_dev, bench_scene, bench_device_scene, bench_sample,
                                    mode, tile):
    torch = torch_dev
    scene, cams = bench_scene
    px, g, ref0, ref = bench_sample
    _say("1.07M-voxel scene sampled parity N=%d, %s, tile %d" % (scene.n_voxels, mode, tile))
    r, rgba, gg, gs, E = _bench_frame(torch, bench_device_scene, cams[0], mode, tile, g)
    err = _check_rgba(rgba.cpu().numpy().astype(np.float64), ref0, pixels=px)
    e1 = _check_grad(gg.cpu().numpy(), ref["grad_grid"], "grad_grid")
    e2 = _check_grad(gs.cpu().numpy(), ref["grad_sh"], "grad_sh")
    _say("  E=%d rgba err %.2e, grad rel err %.2e / %.2e" % (E, err, e1, e2))
    r.release_graph()


def test_forward_invariant_to_sync_mode(torch_dev, bench_scene):
    """The forward has no atomics: the image is bit-identical whether the entry
    count is read back (sort sized to E) or not (sort sized to capacity)."""
    torch = torch_dev
    scene, cams = bench_scene
    a = _gpu_frame(torch, scene, cams, K=2, sync=True)["rgba"]
    b = _gpu_frame(torch, scene, cams, K=2, sync=False)["rgba"]
    assert np.array_equal(a, b)


@pytest.mark.parametrize("mode,tile", [("eager", 16), ("graph", 8)])
def test_bench_scene_sorted_entries_bit_exact(torch_dev, bench_scene, bench_device_scene,
                                              bench_rank_table, mode, tile):
    """The whole sorted list of the benchmark view (1.1-1.7M entries)."""
    torch = torch_dev
    scene, cams = bench_scene
    _say("sorted entries, 1.07M-voxel scene, %s, tile %d" % (mode, tile))
    P = cams[0].W * cams[0].H
    r, _, _, _, E = _bench_frame(torch, bench_device_scene, cams[0], mode, tile,
                                 np.zeros((P, 4)))
    keys, vals = r.sorted_entries(E)
    check_sorted_list(scene, cams[0], keys.cpu().numpy().view(np.uint64),
                      vals.cpu().numpy().view(np.uint32), True, tile=tile,
                      rank_table=bench_rank_table)
    r.release_graph()


def _pixel_roi(scene, cam, voxels, margin=1.5):
    """Pixels whose rays can meet any of `voxels`: the box of the projected
    corners, widened by `margin` pixels (None when a corner is not in front
    of the camera)."""
    R = np.asarray(cam.w2c, np.float64)[:, :3]
    t = np.asarray(cam.w2c, np.float64)[:, 3]
    px = []
    for v in voxels:
        c = scene.center[:, v].astype(np.float64)
        h = 0.5 * float(scene.size[v])
        corners = c + h * np.array([[dx, dy, dz] for dx in (-1, 1) for dy in (-1, 1)
                                    for dz in (-1, 1)], np.float64)
        q = corners @ R.T + t
        if (q[:, 2] <= 1e-3).any():
            return None
        u = cam.fx * q[:, 0] / q[:, 2] + cam.cx
        w = cam.fy * q[:, 1] / q[:, 2] + cam.cy
        x0, x1 = max(0, int(np.floor(u.min() - margin))), min(cam.W - 1, int(np.floor(u.max() + margin)))
        y0, y1 = max(0, int(np.floor(w.min() - margin))), min(cam.H - 1, int(np.floor(w.max() + margin)))
        if x0 > x1 or y0 > y1:
            continue
        yy, xx = np.meshgrid(np.arange(y0, y1 + 1), np.arange(x0, x1 + 1), indexing="ij")
        px.append((yy * cam.W + xx).reshape(-1))
    return np.unique(np.concatenate(px)) if px else np.zeros(0, np.int64)


def test_bench_scene_gradients_against_oracle_central_differences(torch_dev, bench_scene,
                                                                  bench_device_scene):
    """64 sampled parameters of the benchmark view (32 corner raw densities, 32
    SH coefficients; Supp. A.2 gradient of alpha chained through the
    compositing and colour equations): the GPU gradient through
    torch.autograd.Function against the oracle's FP64 adjoint within 1e-3
    relative, and the oracle's adjoint against FP64 central differences of
    the oracle's own render over the parameter's pixel region within 1e-6
    relative.  The upstream gradient is N(0, 1) on the union of the regions
    (zero on pixels the oracle flags) and zero elsewhere, so each sampled
    parameter's gradient is complete on both sides."""
    import dataclasses
    torch = torch_dev
    from paper_2412_04459_amd.render import Rasterizer, render
    scene, cams = bench_scene
    cam = cams[0]
    P = cam.W * cam.H
    ds = bench_device_scene
    _say("oracle central differences, 1.07M-voxel scene")
    rast = Rasterizer(ds, [cam], K=2, tile=8)
    # candidates: parameters with a sizeable gradient under a dense upstream
    # gradient (selection only; the values compared come from the runs below)
    grid = ds.grid_raw.clone().requires_grad_(True)
    sh = ds.sh.clone().requires_grad_(True)
    g0 = torch.from_numpy(S.upstream_grads(P, 21)).cuda()
    (render(rast, grid, sh) * g0).sum().backward()
    gg0 = np.abs(grid.grad.cpu().numpy().astype(np.float64))
    gs0 = np.abs(sh.grad.cpu().numpy().astype(np.float64).reshape(-1))
    del grid, sh
    rng = np.random.default_rng(77)
    vg = scene.vox_grid.reshape(scene.n_voxels, 8)
    slots = np.argsort(vg.reshape(-1), kind="stable")
    starts = np.searchsorted(vg.reshape(-1)[slots], np.arange(scene.n_grid + 1))
    o = cam.position()
    params = []  # (kind, index, voxels)
    for m in rng.permutation(np.nonzero(gg0 > np.median(gg0[gg0 > 0]))[0]):
        vox = slots[starts[m]:starts[m + 1]] // 8
        if _pixel_roi(scene, cam, vox) is not None:
            params.append(("grid", int(m), vox))
        if len(params) == 32:
            break
    for e in rng.permutation(np.nonzero(gs0 > np.median(gs0[gs0 > 0]))[0]):
        v, ch = int(e) // 48, int(e) % 3
        Yv = oracle.sh_basis(3, scene.center[:, v].astype(np.float64) - o)
        pre = float(np.dot(Yv, scene.sh[v, :, ch].astype(np.float64)))
        if abs(pre) > 1e-3 and _pixel_roi(scene, cam, [v]) is not None:
            params.append(("sh", int(e), np.array([v])))
        if len(params) == 64:
            break
    assert len(params) == 64
    rois = [_pixel_roi(scene, cam, vox) for _, _, vox in params]
    union = np.unique(np.concatenate(rois))
    _say("  %d parameters, %d pixels in their regions" % (len(params), len(union)))
    g = np.zeros((P, 4), np.float32)
    g[union] = S.upstream_grads(P, 22)[union]
    flags = oracle.render(scene, cam, K=2, pixels=union)["flags"]
    g[union[flags != 0]] = 0.0
    ref = oracle.render(scene, cam, K=2, pixels=union, grad_rgba=g[union].astype(np.float64))
    grid = ds.grid_raw.clone().requires_grad_(True)
    sh = ds.sh.clone().requires_grad_(True)
    (render(rast, grid, sh) * torch.from_numpy(g).cuda()).sum().backward()
    torch.cuda.synchronize()
    gpu_g = grid.grad.cpu().numpy().astype(np.float64)
    gpu_s = sh.grad.cpu().numpy().astype(np.float64).reshape(-1)
    ref_s = ref["grad_sh"].reshape(-1)
    raw64 = scene.grid_raw.astype(np.float64)
    sh64 = scene.sh.astype(np.float64)
    e_gpu, e_fd = [], []
    for (kind, idx, _), roi in zip(params, rois):
        theta = raw64[idx] if kind == "grid" else sh64.reshape(-1)[idx]
        h = 1e-4 * max(1.0, abs(theta))
        loss = []
        for sgn in (1.0, -1.0):
            if kind == "grid":
                p = raw64.copy(); p[idx] += sgn * h
                sc = dataclasses.replace(scene, grid_raw=p)
            else:
                p = sh64.copy().reshape(-1); p[idx] += sgn * h
                sc = dataclasses.replace(scene, sh=p.reshape(sh64.shape))
            out = oracle.render(sc, cam, K=2, pixels=roi)
            loss.append(float((out["rgba"] * g[roi].astype(np.float64)).sum()))
        fd = (loss[0] - loss[1]) / (2 * h)
        r_o = ref["grad_grid"][idx] if kind == "grid" else ref_s[idx]
        r_g = gpu_g[idx] if kind == "grid" else gpu_s[idx]
        assert r_o != 0.0
        e_fd.append(abs(fd - r_o) / abs(r_o))
        e_gpu.append(abs(r_g - r_o) / abs(r_o))
    e_fd, e_gpu = np.array(e_fd), np.array(e_gpu)
    _say("  oracle adjoint vs oracle FD: max rel %.2e; GPU vs oracle adjoint: max rel %.2e"
         % (e_fd.max(), e_gpu.max()))
    assert e_fd.max() <= 1e-6
    assert e_gpu.max() <= 1e-3


def test_autograd_central_differences_bench_scene(torch_dev, bench_scene, bench_device_scene):
    """fp32 smoke check of the autograd path: gradients from
    torch.autograd through the C ABI against central finite differences of
    the GPU forward on 64 sampled parameters (32 corner raw densities, 32 SH
    coefficients) of the benchmark view, h = 1e-2 max(1, |theta|): the fp32
    rendering error of the affected pixels (about 1e-7 of their values)
    divided by h is the noise of the difference quotient, and at h = 1e-3 it
    reaches 2e-2 of the smallest sampled gradients.  The forward is
    deterministic, so the two perturbed renders differ only where the
    parameter acts; the loss is summed in float64."""
    torch = torch_dev
    from paper_2412_04459_amd.render import Rasterizer, render
    scene, cams = bench_scene
    _say("GPU central differences, 1.07M-voxel scene")
    ds = bench_device_scene
    rast = Rasterizer(ds, cams, K=2)
    grid = ds.grid_raw.clone().requires_grad_(True)
    sh = ds.sh.clone().requires_grad_(True)
    g = torch.from_numpy(S.upstream_grads(cams[0].W * cams[0].H, 21)).cuda()
    rgba = render(rast, grid, sh)
    (rgba * g).sum().backward()
    gg = grid.grad.detach().cpu().numpy().astype(np.float64)
    gs = sh.grad.detach().cpu().numpy().astype(np.float64).reshape(-1)

    def loss(grid_t, sh_t):
        with torch.no_grad():
            out = rast.forward(grid_t, sh_t)
            return float((out.double() * g.double()).sum().item())

    rng = np.random.default_rng(77)
    # grid densities: among the largest gradients
    top = np.argsort(-np.abs(gg))[:2000]
    pick_g = rng.choice(top, 32, replace=False)
    base_grid = ds.grid_raw.clone()
    errs = []
    for m in pick_g:
        h = 1e-2 * max(1.0, abs(float(scene.grid_raw[m])))
        up = base_grid.clone(); up[m] += h
        dn = base_grid.clone(); dn[m] -= h
        fd = (loss(up, ds.sh) - loss(dn, ds.sh)) / (2 * h)
        errs.append(abs(fd - gg[m]) / max(abs(fd), abs(gg[m])))
    # SH coefficients: linear in the coefficient unless the clamp at 0 flips;
    # take channels whose pre-clamp colour is far from 0 (|pre| > 0.05)
    o = cams[0].position()
    top = np.argsort(-np.abs(gs))[:4000]
    ok = []
    for e in top:
        v, ch = int(e) // 48, int(e) % 3
        Yv = oracle.sh_basis(3, scene.center[:, v].astype(np.float64) - o)
        pre = float(np.dot(Yv, scene.sh[v, :, ch].astype(np.float64)))
        if abs(pre) > 0.05:
            ok.append(int(e))
    pick_s = rng.choice(ok, 32, replace=False)
    base_sh = ds.sh.clone().reshape(-1)
    for e in pick_s:
        h = 1e-2 * max(1.0, abs(float(base_sh[e])))
        up = base_sh.clone(); up[e] += h
        dn = base_sh.clone(); dn[e] -= h
        fd = (loss(ds.grid_raw, up.reshape(ds.sh.shape)) - loss(ds.grid_raw, dn.reshape(ds.sh.shape))) / (2 * h)
        errs.append(abs(fd - gs[e]) / max(abs(fd), abs(gs[e])))
    errs = np.array(errs)
    _say("  relative FD error: median %.2e max %.2e" % (np.median(errs), errs.max()))
    assert errs.max() < 1e-2


# ---------------------------------------------------------------------------
# training statistics (Sec. 3.2.2): per-voxel max blending weight (forward)
# and subdivision priority (backward)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("case,K,tile", [("shell_opaque", 2, 16), ("shell", 1, 8),
                                         ("tiny", 3, 8)])
def test_training_statistics_match_oracle(torch_dev, case, K, tile):
    torch = torch_dev
    from paper_2412_04459_amd.render import DeviceScene, Rasterizer
    if case.startswith("shell"):
        scene, cams = S.sphere_shell_scene(opaque=case.endswith("opaque")), [S.sphere_shell_camera()]
    else:
        scene = S.tiny_random_scene(9, max_level=4, sh_degree=3)
        cams = [S.look_at(90, 70, 80.0, [1.7, 1.4, 1.2], target=(0.5, 0.5, 0.5))]
    _say("training statistics %s K=%d tile %d" % (case, K, tile))
    P = cams[0].W * cams[0].H
    g = S.upstream_grads(P, 8)
    ref0 = oracle.render(scene, cams[0], K=K)
    flagged = ref0["flags"] != 0
    g[flagged] = 0.0
    ref = oracle.render(scene, cams[0], K=K, grad_rgba=g.astype(np.float64), train_stats=True)
    # max weight over the unflagged pixels only: the GPU may decide a
    # termination band either way, so its maximum lies between the two
    ref_u = oracle.render(scene, cams[0], K=K, pixels=np.nonzero(~flagged)[0], train_stats=True)
    ds = DeviceScene(scene)
    rast = Rasterizer(ds, cams, K=K, tile=tile)
    mw = torch.zeros(scene.n_voxels, dtype=torch.float32, device="cuda")
    pr = torch.zeros(scene.n_voxels, dtype=torch.float32, device="cuda")
    rast.forward(max_weight=mw)
    gt = torch.from_numpy(g).cuda()
    rast.backward(gt, priority=pr)
    torch.cuda.synchronize()
    m = mw.cpu().numpy().astype(np.float64)
    lo = np.minimum(ref["max_weight"], ref_u["max_weight"])
    hi = np.maximum(ref["max_weight"], ref_u["max_weight"])
    assert (m >= lo - RGBA_TOL).all() and (m <= hi + RGBA_TOL).all(), \
        "max weight off by %.3g" % max((lo - m).max(), (m - hi).max())
    assert (ref["max_weight"] > 0).sum() > 10
    _check_grad(pr.cpu().numpy().astype(np.float64), ref["priority"], "priority")
    # statistics accumulate across calls: the maximum stays, the sum doubles
    rast.forward(max_weight=mw)
    rast.backward(gt, priority=pr)
    torch.cuda.synchronize()
    assert np.array_equal(mw.cpu().numpy().astype(np.float64), m)
    _check_grad(pr.cpu().numpy().astype(np.float64), 2 * ref["priority"], "priority x2")


def test_training_statistics_leave_image_and_gradients_unchanged(torch_dev):
    torch = torch_dev
    from paper_2412_04459_amd.render import DeviceScene, Rasterizer
    scene, cams = S.sphere_shell_scene(opaque=True), [S.sphere_shell_camera()]
    ds = DeviceScene(scene)
    rast = Rasterizer(ds, cams, K=2, tile=8)
    g = torch.from_numpy(S.upstream_grads(cams[0].W * cams[0].H, 9)).cuda()
    a = rast.forward().clone()
    ga, sa = [t.clone() for t in rast.backward(g)]
    mw = torch.zeros(scene.n_voxels, dtype=torch.float32, device="cuda")
    pr = torch.zeros_like(mw)
    b = rast.forward(max_weight=mw)
    gb, sb = rast.backward(g, priority=pr)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    # gradients go through float atomics: equal up to summation order
    assert torch.allclose(ga, gb, rtol=1e-5, atol=1e-7) and torch.allclose(sa, sb, rtol=1e-5, atol=1e-7)


# ---------------------------------------------------------------------------
# depth and normal images (Sec. 3.1.1 "Voxel normal", "Voxel depth") and
# their adjoint
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("case,K,act,tile", [("shell_opaque", 2, 0, 16), ("shell", 3, 0, 8),
                                             ("tiny", 2, 1, 8), ("shell_opaque", 1, 0, 32)])
def test_depth_normal_match_oracle(torch_dev, case, K, act, tile):
    torch = torch_dev
    from paper_2412_04459_amd.render import DeviceScene, Rasterizer
    if case.startswith("shell"):
        scene, cams = S.sphere_shell_scene(opaque=case.endswith("opaque")), [S.sphere_shell_camera()]
    else:
        scene = S.tiny_random_scene(9, max_level=4, sh_degree=3)
        cams = [S.look_at(90, 70, 80.0, [1.7, 1.4, 1.2], target=(0.5, 0.5, 0.5))]
    _say("depth and normal %s K=%d act=%d tile %d" % (case, K, act, tile))
    P = cams[0].W * cams[0].H
    rng = np.random.default_rng(40 + K)
    g = S.upstream_grads(P, 10)
    gd = rng.normal(size=P).astype(np.float32)
    gn = rng.normal(size=(P, 3)).astype(np.float32)
    ref0 = oracle.render(scene, cams[0], K=K, activation=act, depth_normal=True)
    ok = ref0["flags"] == 0
    g[~ok] = 0.0
    gd[~ok] = 0.0
    gn[~ok] = 0.0
    ref = oracle.render(scene, cams[0], K=K, activation=act, grad_rgba=g.astype(np.float64),
                        depth_normal=True, grad_depth=gd.astype(np.float64),
                        grad_normal=gn.astype(np.float64))
    ds = DeviceScene(scene)
    rast = Rasterizer(ds, cams, K=K, activation=act, tile=tile)
    dep = torch.empty(P, dtype=torch.float32, device="cuda")
    nrm = torch.empty((P, 3), dtype=torch.float32, device="cuda")
    rgba = rast.forward(depth=dep, normal=nrm)
    gg, gs = rast.backward(torch.from_numpy(g).cuda(), grad_depth=torch.from_numpy(gd).cuda(),
                           grad_normal=torch.from_numpy(gn).cuda())
    torch.cuda.synchronize()
    _check_rgba(rgba.cpu().numpy().astype(np.float64), ref0)
    d = dep.cpu().numpy().astype(np.float64)
    n = nrm.cpu().numpy().astype(np.float64)
    ed = np.abs(d - ref0["depth"])[ok]
    en = np.abs(n - ref0["normal"]).max(1)[ok]
    assert ed.max() <= RGBA_TOL * max(1.0, np.abs(ref0["depth"]).max()), "depth off by %.3g" % ed.max()
    assert en.max() <= RGBA_TOL, "normal off by %.3g" % en.max()
    assert np.abs(ref0["depth"]).max() > 0.1 and np.abs(ref0["normal"]).max() > 0.01
    _check_grad(gg.cpu().numpy().astype(np.float64), ref["grad_grid"], "grad_grid")
    _check_grad(gs.cpu().numpy().astype(np.float64), ref["grad_sh"], "grad_sh")


# ---------------------------------------------------------------------------
# anti-aliasing (Sec. 3.1.2): supersampled render, anti-aliased downsample,
# background colour; and the adjoint
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("src,dst", [((71, 53), (64, 48)), ((96, 96), (64, 64)),
                                     ((128, 90), (64, 45)), ((31, 17), (31, 17)),
                                     ((1412, 924), (1284, 840))])
def test_downsample_and_adjoint_match_oracle(torch_dev, src, dst):
    torch = torch_dev
    from paper_2412_04459_amd.render import downsample
    rng = np.random.default_rng(src[0] + dst[1])
    bg = [0.25, 0.5, 0.75]
    x = rng.random((src[1], src[0], 4)).astype(np.float32)
    y = rng.normal(size=(dst[1], dst[0], 4)).astype(np.float32)
    xt = torch.from_numpy(x.reshape(-1, 4)).cuda().requires_grad_(True)
    out = downsample(xt, src[0], src[1], dst[0], dst[1], bg)
    (out * torch.from_numpy(y.reshape(-1, 4)).cuda()).sum().backward()
    torch.cuda.synchronize()
    ref = oracle.downsample(x.astype(np.float64), dst[0], dst[1], bg)
    assert np.abs(out.detach().cpu().numpy().reshape(ref.shape) - ref).max() <= 1e-5
    gref = oracle.downsample_adjoint(y.astype(np.float64), src[0], src[1], bg)
    g = xt.grad.cpu().numpy().reshape(gref.shape)
    assert np.abs(g - gref).max() <= 1e-5 * max(1.0, np.abs(gref).max())


def test_supersampled_render_with_background_matches_oracle(torch_dev):
    """The view rendered at 1.5x, downsampled with the tent filter and given a
    background colour; gradients through both (autograd) against the oracle's
    render at 1.5x with the oracle's transpose of the filter."""
    torch = torch_dev
    from paper_2412_04459_amd.render import (DeviceScene, Rasterizer, downsample, render,
                                              supersampled_camera)
    scene, cam = S.sphere_shell_scene(opaque=True), S.sphere_shell_camera()
    hi = supersampled_camera(cam, 1.5)
    assert (hi.W, hi.H) == (96, 96)
    bg = [0.2, 0.3, 0.4]
    ds = DeviceScene(scene)
    rast = Rasterizer(ds, [hi], K=2, tile=8)
    grid = ds.grid_raw.clone().requires_grad_(True)
    sh = ds.sh.clone().requires_grad_(True)
    img = downsample(render(rast, grid, sh), hi.W, hi.H, cam.W, cam.H, bg)
    g = S.upstream_grads(cam.W * cam.H, 11)
    ref_hi = oracle.render(scene, hi, K=2)
    # pixels of the low-res image whose filter taps reach a flagged pixel
    flag_lo = oracle.downsample(np.repeat((ref_hi["flags"] != 0).astype(np.float64), 4)
                                .reshape(hi.H, hi.W, 4), cam.W, cam.H)[..., 0] > 0
    g[flag_lo.reshape(-1)] = 0.0
    (img * torch.from_numpy(g).cuda()).sum().backward()
    torch.cuda.synchronize()
    ref_img = oracle.downsample(ref_hi["rgba"].reshape(hi.H, hi.W, 4), cam.W, cam.H, bg)
    err = np.abs(img.detach().cpu().numpy().reshape(ref_img.shape) - ref_img).max(-1)
    assert err[~flag_lo].max() <= RGBA_TOL
    g_hi = oracle.downsample_adjoint(g.reshape(cam.H, cam.W, 4).astype(np.float64), hi.W, hi.H, bg)
    ref = oracle.render(scene, hi, K=2, grad_rgba=g_hi.reshape(-1, 4))
    _check_grad(grid.grad.cpu().numpy().astype(np.float64), ref["grad_grid"], "grad_grid")
    _check_grad(sh.grad.cpu().numpy().astype(np.float64), ref["grad_sh"], "grad_sh")


def test_autograd_backward_after_a_second_render(torch_dev):
    """Two renders through the same rasterizer before backward (two loss
    terms over different densities): each output's gradient equals the
    gradient of a single forward/backward with its own parameters."""
    torch = torch_dev
    from paper_2412_04459_amd.render import DeviceScene, Rasterizer, render
    scene = S.sphere_shell_scene(opaque=True)
    cams = [S.sphere_shell_camera()]
    ds = DeviceScene(scene)
    rast = Rasterizer(ds, cams, K=2, tile=8)
    P = cams[0].W * cams[0].H
    ga = torch.from_numpy(S.upstream_grads(P, 41)).cuda()
    gb = torch.from_numpy(S.upstream_grads(P, 42)).cuda()
    raw_b = (ds.grid_raw * 0.5 - 0.3).contiguous()
    # references: one frame each
    ref_a = rast.forward(ds.grid_raw, ds.sh).clone()
    a_gg, a_gs = [t.clone() for t in rast.backward(ga, ds.grid_raw, ds.sh)]
    rast.forward(raw_b, ds.sh)
    b_gg, b_gs = [t.clone() for t in rast.backward(gb, raw_b, ds.sh)]
    # both renders first, then one backward over both loss terms
    grid_a = ds.grid_raw.clone().requires_grad_(True)
    grid_b = raw_b.clone().requires_grad_(True)
    sh = ds.sh.clone().requires_grad_(True)
    out_a = render(rast, grid_a, sh)
    out_b = render(rast, grid_b, sh)
    assert torch.equal(out_a, ref_a)
    ((out_a * ga).sum() + (out_b * gb).sum()).backward()
    torch.cuda.synchronize()
    assert torch.allclose(grid_a.grad, a_gg, rtol=1e-5, atol=1e-7)
    assert torch.allclose(grid_b.grad, b_gg, rtol=1e-5, atol=1e-7)
    assert torch.allclose(sh.grad, a_gs + b_gs, rtol=1e-5, atol=1e-6)


# ---------------------------------------------------------------------------
# the large scene (about 8M voxels, max level 14, SH degree 3, K = 1) at one
# 1920x1080 view of its orbit, 8x8 tiles, no host synchronisation, one
# captured hipGraph: sampled pixels and gradients against the oracle, and
# the sorted lists of sampled tiles bit-exact
# ---------------------------------------------------------------------------
def test_large_scene_view_sampled_parity(torch_dev):
    torch = torch_dev
    from paper_2412_04459_amd.render import DeviceScene, zcurve_relabel
    scene, _ = zcurve_relabel(S.large_shells_scene())
    cam = S.orbit_cameras_1080p()[0]
    P = cam.W * cam.H
    _say("large scene N=%d, one 1920x1080 view" % scene.n_voxels)
    ds = DeviceScene(scene)
    # sample: pixels with hits (from an untimed frame) and random pixels
    _, rgba0, _, _, _ = _large_frame(torch, ds, cam, np.zeros((P, 4), np.float32))
    a0 = rgba0[:, 3].cpu().numpy()
    rng = np.random.default_rng(17)
    px = np.unique(np.concatenate([rng.choice(np.nonzero(a0 > 0)[0], 300, replace=False),
                                   rng.choice(P, 60, replace=False)]))
    ref0 = oracle.render(scene, cam, K=1, pixels=px)
    g = np.zeros((P, 4), np.float32)
    g[px] = S.upstream_grads(P, 4)[px]
    g[px[ref0["flags"] != 0]] = 0.0
    ref = oracle.render(scene, cam, K=1, pixels=px, grad_rgba=g[px].astype(np.float64))
    r, rgba, gg, gs, E = _large_frame(torch, ds, cam, g)
    _check_rgba(rgba.cpu().numpy().astype(np.float64), ref0, pixels=px)
    _check_grad(gg.cpu().numpy(), ref["grad_grid"], "grad_grid")
    _check_grad(gs.cpu().numpy(), ref["grad_sh"], "grad_sh")
    # sorted lists of sampled tiles: every entry's key and value against the
    # oracle's, each tile's entries strictly ascending in the paper's key
    # order, and the tile's entry set between the oracle's bounds
    keys, vals = r.sorted_entries(E)
    gk = keys.cpu().numpy().view(np.uint64)
    gv = vals.cpu().numpy().view(np.uint32)
    key_low = int(8 * scene.n_voxels - 1).bit_length()
    assert np.all(gk[1:] > gk[:-1])
    tid = (gk >> np.uint64(key_low)).astype(np.int64)
    ntile = ((cam.W + 7) // 8) * ((cam.H + 7) // 8)
    pick = rng.choice(np.unique(tid), 40, replace=False)
    sel = np.isin(tid, pick)
    vid = (gv[sel] & np.uint32((1 << 29) - 1)).astype(np.int64)
    sgn = (gv[sel] >> np.uint32(29)).astype(np.uint8)
    _, kc, val = oracle.keys(tid[sel], vid, sgn, scene.octpath, scene.max_level)
    assert np.array_equal(val, gv[sel])
    for t in pick:
        kt = kc[tid[sel] == t]
        assert np.all(kt[1:] > kt[:-1]), "tile %d out of the paper's key order" % t
    # the low key bits are the rank of (path XOR s, s) among all 8N pairs
    n8 = 8 * scene.n_voxels
    all_vid = np.repeat(np.arange(scene.n_voxels, dtype=np.int64), 8)
    all_sgn = np.tile(np.arange(8, dtype=np.uint8), scene.n_voxels)
    _, all_kc, _ = oracle.keys(np.zeros(n8, np.int64), all_vid, all_sgn, scene.octpath,
                               scene.max_level)
    del all_vid, all_sgn
    all_kc.sort()
    _, own, _ = oracle.keys(np.zeros(vid.size, np.int64), vid, sgn, scene.octpath, scene.max_level)
    rank = np.searchsorted(all_kc, own)
    del all_kc
    low = (gk[sel] & np.uint64((1 << key_low) - 1)).astype(np.int64)
    assert np.array_equal(low, rank)
    exp = oracle.expected_entries(scene, cam, tile_w=8, tile_h=8)
    for name, bound in (("must", exp["must"]), ("may", exp["may"])):
        bk = bound[0]
        btile = (bk >> np.uint64(3 * scene.max_level + 3)).astype(np.int64)
        inb = bk[np.isin(btile, pick)]
        if name == "must":
            assert np.all(np.isin(inb, kc)), "missing required entries"
            assert inb.size > 0
        else:
            assert np.all(np.isin(kc, inb)), "entries outside the band"
    assert tid.max() < ntile
    r.release_graph()


def _large_frame(torch, ds, cam, grad):
    """One fwd+bwd frame of a 1920x1080 view of the large scene, K = 1, in the
    batched benchmark's configuration (8x8 tiles, capacity from a counted
    probe, no host synchronisation, captured hipGraph)."""
    from paper_2412_04459_amd.render import Rasterizer
    probe = Rasterizer(ds, [cam], K=1, sync_count=True, tile=8)
    probe.preprocess()
    cap = int(probe.n_entries * 1.1) + 4096
    del probe
    r = Rasterizer(ds, [cam], K=1, capacity=cap, sync_count=False, tile=8)
    P = cam.W * cam.H
    g = torch.from_numpy(np.ascontiguousarray(grad, np.float32)).cuda()
    rgba = torch.empty((P, 4), dtype=torch.float32, device="cuda")
    gg = torch.empty((ds.n_grid,), dtype=torch.float32, device="cuda")
    gs = torch.empty_like(ds.sh)
    stream = torch.cuda.Stream()
    r.capture(rgba, g, gg, gs, stream)
    r.replay(stream)
    torch.cuda.synchronize()
    E = r.check_overflow()
    assert 0 < E <= cap
    return r, rgba, gg, gs, E
