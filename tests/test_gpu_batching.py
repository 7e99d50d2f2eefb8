"""GPU tests of the batched form: several cameras of uneven size in one launch
per stage, runtime tile edge, persistent scheduling, hipGraph replay.

The forward has no atomics and every pixel runs the same operation sequence
whatever the tiling or batching, so images must be bit-identical across those
settings; gradients (float atomics) agree to tolerance.
"""
import numpy as np
import pytest

import oracle
from paper_2412_04459_amd import scenes as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _say(msg):
    print(msg, flush=True)


def _grad_close(a, b, rel=1e-4, floor=1e-6):
    a = a.detach().cpu().double().numpy().reshape(-1)
    b = b.detach().cpu().double().numpy().reshape(-1)
    tol = rel * np.abs(b) + floor * np.abs(b).max()
    return bool(np.all(np.abs(a - b) <= tol))


def _scene_and_cams():
    scene = S.sphere_shell_scene(opaque=True)
    cams = [S.look_at(64, 64, 50.0, [1.6, 1.0, 0.9], target=(0.25, 0.25, 0.25)),
            S.look_at(77, 51, 60.0, [1.5, -1.2, 1.0], target=(0.3, 0.3, 0.3)),
            S.look_at(40, 96, 55.0, [-0.8, 1.7, 1.2], target=(0.2, 0.3, 0.25))]
    return scene, cams


@pytest.mark.parametrize("tile,persistent", [(16, 0), (8, 0), (32, 0), (16, 64), (8, 96), (32, 7)])
def test_tile_and_schedule_invariance(torch_dev, tile, persistent):
    torch = torch_dev
    from paper_2412_04459_amd.render import DeviceScene, Rasterizer
    scene, cams = _scene_and_cams()
    _say("tile=%d persistent=%d" % (tile, persistent))
    ds = DeviceScene(scene)
    ref = Rasterizer(ds, cams[:1], K=2)
    a = ref.forward().cpu().numpy()
    r = Rasterizer(ds, cams[:1], K=2, tile=tile, persistent=persistent)
    b = r.forward().cpu().numpy()
    assert np.array_equal(a, b)
    g = torch.from_numpy(S.upstream_grads(a.shape[0], 4)).cuda()
    ga, sa = ref.backward(g)
    gb, sb = r.backward(g)
    torch.cuda.synchronize()
    assert _grad_close(gb, ga) and _grad_close(sb, sa)
    # and against the oracle
    o = oracle.render(scene, cams[0], K=2)
    err = np.minimum(np.abs(b - o["rgba"]).max(1), np.abs(b - o["rgba_alt"]).max(1))
    assert err.max() <= 1e-4


def test_batched_cameras_equal_single_views(torch_dev):
    torch = torch_dev
    from paper_2412_04459_amd.render import DeviceScene, Rasterizer
    scene, cams = _scene_and_cams()
    ds = DeviceScene(scene)
    rb = Rasterizer(ds, cams, K=1)
    big = rb.forward().cpu().numpy()
    P = [c.W * c.H for c in cams]
    g = torch.from_numpy(S.upstream_grads(sum(P), 6)).cuda()
    gg_b, gs_b = rb.backward(g)
    off = 0
    gg_sum = torch.zeros_like(gg_b)
    gs_sum = torch.zeros_like(gs_b)
    for c, p in zip(cams, P):
        r = Rasterizer(ds, [c], K=1)
        one = r.forward().cpu().numpy()
        assert np.array_equal(one, big[off:off + p])
        a, b = r.backward(g[off:off + p].contiguous())
        gg_sum += a
        gs_sum += b
        off += p
    torch.cuda.synchronize()
    assert _grad_close(gg_b, gg_sum) and _grad_close(gs_b, gs_sum)


def test_graph_replays_match_eager(torch_dev):
    torch = torch_dev
    from paper_2412_04459_amd.render import DeviceScene, Rasterizer
    scene, cams = _scene_and_cams()
    ds = DeviceScene(scene)
    eager = Rasterizer(ds, cams, K=2, tile=8)
    rgba_e = eager.forward()
    P = rgba_e.shape[0]
    g = torch.from_numpy(S.upstream_grads(P, 8)).cuda()
    gg_e, gs_e = eager.backward(g)
    torch.cuda.synchronize()
    r = Rasterizer(ds, cams, K=2, tile=8, persistent=32, sync_count=False,
                   capacity=eager.n_entries + 1000)
    rgba = torch.full_like(rgba_e, -1.0)
    gg = torch.full_like(gg_e, 7.0)
    gs = torch.full_like(gs_e, 7.0)
    stream = torch.cuda.Stream()
    r.capture(rgba, g, gg, gs, stream)
    for rep in range(3):
        rgba.fill_(-1.0)
        gg.fill_(7.0)
        gs.fill_(7.0)
        torch.cuda.synchronize()
        r.replay(stream)
        torch.cuda.synchronize()
        assert torch.equal(rgba, rgba_e), "replay %d" % rep
        assert _grad_close(gg, gg_e) and _grad_close(gs, gs_e), "replay %d" % rep
        # unrelated eager work between replays
        eager.forward()
        torch.cuda.synchronize()
    assert r.check_overflow() <= r.capacity
    r.release_graph()


@pytest.mark.parametrize("group", [1, 2, 3])
def test_batch_renderer_groups(torch_dev, group):
    torch = torch_dev
    from paper_2412_04459_amd.render import BatchRenderer, DeviceScene, Rasterizer
    scene, cams = _scene_and_cams()
    ds = DeviceScene(scene)
    ref = Rasterizer(ds, cams, K=2)
    a = ref.forward()
    g = torch.from_numpy(S.upstream_grads(a.shape[0], 9)).cuda()
    ga, sa = ref.backward(g)
    br = BatchRenderer(ds, cams, K=2, group=group, tile=16, persistent=0)
    br.capture(g)
    br.replay()
    torch.cuda.synchronize()
    assert torch.equal(br.rgba, a)
    assert _grad_close(br.grad_grid, ga) and _grad_close(br.grad_sh, sa)
    assert br.check_overflow()


def test_autotuner_runs_and_picks_a_measured_candidate(torch_dev):
    torch = torch_dev
    from paper_2412_04459_amd.autotune import tune
    from paper_2412_04459_amd.render import DeviceScene
    scene, cams = _scene_and_cams()
    ds = DeviceScene(scene)
    P = sum(c.W * c.H for c in cams)
    g = torch.from_numpy(S.upstream_grads(P, 10)).cuda()
    res = tune(ds, cams, 2, g, tiles=(8, 16), persistent=(0, 64), reps=2)
    assert res["tile"] in (8, 16) and res["group"] in (1, 2, 3)
    assert any(r["tile"] == res["tile"] and r["group"] == res["group"] and
               r["persistent"] == res["persistent"] for r in res["table"])


def test_grid_adjacency_and_gather_path(torch_dev):
    """The corner adjacency lists, for every grid point, exactly the corner
    slots that reference it (increasing); the gather path of the grid gradient
    equals the atomic path to rounding (the per-voxel corner gradients still
    come from float atomics, so neither is bit-reproducible run to run)."""
    torch = torch_dev
    from paper_2412_04459_amd.render import DeviceScene, Rasterizer
    scene = S.spheres_plane_scene()
    cam = S.spheres_plane_camera()
    ds = DeviceScene(scene, grid_adjacency=True)
    off = ds.adj_off.cpu().numpy().astype(np.int64)
    adj = ds.adj.cpu().numpy().astype(np.int64)
    vg = scene.vox_grid.reshape(-1).astype(np.int64)
    order = np.argsort(vg, kind="stable")
    assert off[0] == 0 and off[-1] == vg.size
    assert np.array_equal(adj, order)
    assert np.array_equal(np.diff(off), np.bincount(vg, minlength=scene.n_grid))
    g = torch.from_numpy(S.upstream_grads(cam.W * cam.H, 11)).cuda()
    r1 = Rasterizer(ds, [cam], K=1)
    r1.forward()
    ga, sa = r1.backward(g)
    gb, sb = r1.backward(g)
    torch.cuda.synchronize()
    assert _grad_close(ga, gb)
    ds_atomic = DeviceScene(scene, grid_adjacency=False)
    r2 = Rasterizer(ds_atomic, [cam], K=1)
    r2.forward()
    gc, sc = r2.backward(g)
    torch.cuda.synchronize()
    assert _grad_close(ga, gc) and _grad_close(sa, sc)


def test_batched_wide_tile_ids_match_oracle(torch_dev):
    """Six 1920x1080 cameras in one frame at 8x8 tiles: 194,400 global tile
    ids, so the key's tile field needs 18 bits, beyond the 16 bits of one view
    (Supp. B.1 key layout).  Each camera's block of the sorted list is checked
    bit-exact against the oracle's keys with that camera's tile offset; rgba
    on sampled pixels of every camera and the gradients of an upstream
    gradient on those pixels against the oracle, in the no-sync graph mode
    the batched benchmark uses."""
    torch = torch_dev
    from paper_2412_04459_amd.render import DeviceScene, Rasterizer
    from parity_helpers import (check_grad, check_rgba, check_sorted_list, cpu_order_ranks,
                                key_low_bits)
    scene = S.sphere_shell_scene(opaque=True)
    rng = np.random.default_rng(61)
    cams = [S.look_at(1920, 1080, 50.0, (1.7 + 0.1 * i) * S.random_direction(rng))
            for i in range(6)]
    tiles = [((c.W + 7) // 8) * ((c.H + 7) // 8) for c in cams]
    offs = np.concatenate([[0], np.cumsum(tiles)])
    assert offs[-1] > 1 << 17
    _say("batched wide tile ids: %d cameras, %d tiles" % (len(cams), offs[-1]))
    P = [c.W * c.H for c in cams]
    poff = np.concatenate([[0], np.cumsum(P)])
    # sampled pixels per camera, the oracle's rgba and gradients there
    g = np.zeros((poff[-1], 4), np.float32)
    gfull = S.upstream_grads(int(poff[-1]), 62)
    refs, samples = [], []
    ref_gg = np.zeros(scene.n_grid)
    ref_gs = np.zeros(scene.sh.shape)
    for i, c in enumerate(cams):
        px = np.unique(rng.choice(P[i], 400, replace=False))
        r0 = oracle.render(scene, c, K=2, pixels=px)
        gi = gfull[poff[i] + px].copy()
        gi[r0["flags"] != 0] = 0.0
        g[poff[i] + px] = gi
        rg = oracle.render(scene, c, K=2, pixels=px, grad_rgba=gi.astype(np.float64))
        ref_gg += rg["grad_grid"]
        ref_gs += rg["grad_sh"]
        refs.append(r0)
        samples.append(px)
    ds = DeviceScene(scene)
    probe = Rasterizer(ds, cams, K=2, sync_count=True, tile=8)
    probe.preprocess()
    cap = int(probe.n_entries * 1.1) + 4096
    del probe
    r = Rasterizer(ds, cams, K=2, capacity=cap, sync_count=False, tile=8)
    rgba = torch.full((int(poff[-1]), 4), -1.0, dtype=torch.float32, device="cuda")
    gg = torch.full((ds.n_grid,), 7.0, dtype=torch.float32, device="cuda")
    gs = torch.full_like(ds.sh, 7.0)
    stream = torch.cuda.Stream()
    r.capture(rgba, torch.from_numpy(g).cuda(), gg, gs, stream)
    r.replay(stream)
    torch.cuda.synchronize()
    E = r.check_overflow()
    assert 0 < E <= cap
    keys, vals = r.sorted_entries(E)
    gk = keys.cpu().numpy().view(np.uint64)
    gv = vals.cpu().numpy().view(np.uint32)
    tid = (gk >> np.uint64(key_low_bits(scene, True))).astype(np.int64)
    assert tid.max() >= 1 << 16
    table = cpu_order_ranks(scene)
    out = rgba.cpu().numpy().astype(np.float64)
    for i, c in enumerate(cams):
        sel = (tid >= offs[i]) & (tid < offs[i + 1])
        assert sel.any()
        check_sorted_list(scene, c, gk[sel], gv[sel], True, tile=8, tile_offset=int(offs[i]),
                          rank_table=table)
        check_rgba(out[poff[i]:poff[i + 1]], refs[i], pixels=samples[i])
    assert np.count_nonzero((tid < 0) | (tid >= offs[-1])) == 0
    check_grad(gg.cpu().numpy(), ref_gg, "grad_grid")
    check_grad(gs.cpu().numpy(), ref_gs, "grad_sh")
    r.release_graph()
