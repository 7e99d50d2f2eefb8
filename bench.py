"""Benchmark: forward + backward frames of the sparse-voxel rasterizer on one GPU.

Workload: the ~1.07M-voxel synthetic scene (max level 12, SH degree 3, K = 2
samples per segment, explin) rendered at 1297x840 from a seeded 36-view orbit,
one view per step; a step is the whole hot path for that view:
svr_preprocess (projection, pre-process, duplication), svr_sort, svr_render_fwd
and svr_render_bwd (adjoint into grid densities and SH coefficients).  Inputs
(scene, upstream gradients) are resident in HBM before the timed region.

Prints one JSON line: Mpix/s (pixels x frames / s), frames/s, per-kernel
times measured with HIP events on the launch stream, the roofline of the
dominant kernel, the frame-level HBM fraction, and the FP64 CPU oracle timed
on a bounded pixel sample of the same view.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "fwd+bwd Mpix/s and frames/s at 1M voxels 1297×840; achieved HBM GB/s vs peak"
HBM_PEAK_GBS = 8000.0
# VALU issue peak of MI355X without packed fp32: 256 CUs x 4 SIMDs x 16 lanes
# x 2.4 GHz = 39.3e12 lane operations per second.
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# Algorithmic VALU lane operations of the render kernels, two counts.
# "design": the operations the kernels' inner loops perform, counted per
# walked (pixel, entry) pair and per hit from the code's arithmetic (sign
# test + fp64 slab test per pair; K samples of local coordinate, trilinear,
# activation, then alpha and compositing per hit; the backward recomputes the
# forward's hit and forms the 8 corner weights per sample).
# "estimate": the coarser per-unit figures of the measurement plan (about 20
# per pair, 70 + 60 K per forward hit, 2.5 times that per backward hit).
OPS = {
    "design": {"pair": 23, "hit_fwd": lambda K: 13 + 28 * K,
               "hit_bwd": lambda K: 2 * (13 + 28 * K) + 20 * K + 30},
    "estimate": {"pair": 20, "hit_fwd": lambda K: 70 + 60 * K,
                 "hit_bwd": lambda K: 2.5 * (70 + 60 * K)},
}
OPS_PAIR = OPS["design"]["pair"]
OPS_HIT_FWD = OPS["design"]["hit_fwd"]
OPS_HIT_BWD = OPS["design"]["hit_bwd"]
# the paper's forward rendering rate on its RTX 3090 Ti (Mip-NeRF360 at 1x:
# 121 FPS at 1-1.6 Mpix per frame), context only
PAPER_CONTEXT = {"fps": 121, "mpix_s_range": [121, 194], "hardware": "NVIDIA RTX 3090 Ti",
                 "what": "forward rendering only, trained Mip-NeRF360 scenes at 1x evaluation "
                         "resolution (Sec. 4 main results)"}


def frame_bytes(N, Nv, E, P, S):
    """Algorithmic HBM bytes of one fwd+bwd frame, per stage."""
    return {
        "project": 16 * N + 12 * N,                      # centre+size read; count+rect written
        "preprocess": Nv * (32 + 32 + 4 * S + 64),       # indices, densities, SH read; record written
        "emit": E * 12 + Nv * 8,                         # key+value written; path read
        "sort": E * 24,                                  # one read and one write of the list
        "render_fwd": E * 4 + Nv * 72 + P * 24,          # values, records+rects; rgba, tau, last
        "render_bwd": E * 4 + Nv * 72 + P * 24 + Nv * 44,  # + upstream grads; 11 gradients/voxel
        "sh_bwd": N * 4 * S + Nv * (12 + 32 + 32 + 32),  # grad_sh written; colour grads, indices, corner grads
    }


STAGES = [("H1 tile masks + summed-area table", ("tile_masks", "tile_sat"), None),
          ("H2-H3 project + per-view record", ("project",), ("project", "preprocess")),
          ("H4 scan + emit", ("scan_top", "emit", "emit_big"), ("emit",)),
          ("H5-H6 sort + tile ranges", ("sort_hist", "sort_hist_scan", "sort_pass", "tile_count",
                                        "tile_ranges", "tile_place", "tile_order", "tile_sort_small",
                                        "tile_sort_big"),
           ("sort",)),
          ("H7 render forward", ("render_fwd",), ("render_fwd",)),
          ("H8 render backward", ("render_bwd",), ("render_bwd",)),
          ("H9 pre-process adjoint", ("sh_bwd", "grid_gather"), ("sh_bwd",)),
          ("fills", ("fill",), None)]


def stage_rows(per_kernel, N, Nv, E, P, S):
    """Per stage of the path: time per frame (HIP events), algorithmic bytes,
    and the HBM rate those bytes imply against the 8 TB/s peak."""
    fb = frame_bytes(N, Nv, E, P, S)
    rows = {}
    for name, kernels, parts in STAGES:
        ms = sum(per_kernel[k]["ms_per_step"] for k in kernels if k in per_kernel)
        row = {"kernels": list(kernels), "ms_per_step": ms}
        if parts:
            b = float(sum(fb[x] for x in parts))
            row["bytes"] = b
            row["achieved_GBs"] = b / (ms / 1e3) / 1e9 if ms > 0 else None
            row["frac_hbm"] = row["achieved_GBs"] / HBM_PEAK_GBS if ms > 0 else None
        rows[name] = row
    return rows


def kernel_bytes(name, N, Nv, E, P, S, passes):
    if name == "sort_pass":
        return 24 * E / 1.0  # per pass launch: read + write of the list
    fb = frame_bytes(N, Nv, E, P, S)
    return {"project": fb["project"] + fb["preprocess"], "emit": fb["emit"],
            "render_fwd": fb["render_fwd"], "render_bwd": fb["render_bwd"],
            "sh_bwd": fb["sh_bwd"]}.get(name)


def cpu_baseline(scene, cam, K, seconds_target=15.0, threads=None):
    import oracle
    threads = threads or len(os.sched_getaffinity(0))
    rng = np.random.default_rng(99)
    P = cam.W * cam.H
    n = 64
    t_used = 0.0
    done = 0
    if threads == 1:
        n = 16
    while t_used < seconds_target and done < 8192:
        px = rng.choice(P, n, replace=False)
        g = np.random.default_rng(done).normal(size=(n, 4))
        t0 = time.perf_counter()
        oracle.render(scene, cam, K=K, pixels=px, grad_rgba=g, nthreads=threads)
        t_used += time.perf_counter() - t0
        done += n
        n = min(2 * n, 1024 if threads > 1 else 128)
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": done / t_used / 1e6, "unit": "Mpix/s", "cores": threads, "kind": "oracle",
            "sample": "%d seeded pixels of view 0, FP64 brute-force fwd+bwd over all %d voxels "
                      "(%.1f s; CPU: %s)" % (done, scene.n_voxels, t_used, model)}


def kernel_symbol(kind, tile, K, act=0):
    """Name rocprofv3 gives the render kernel instantiation the library
    launches for this tile size, K (templated for K <= 3) and activation."""
    kt = K if K <= 3 else 0
    if kind == "render_fwd":
        return "k_render_fwd<%d, %d, %d, false, false>" % (tile, kt, act)
    if kind == "render_bwd":
        return "k_render_bwd<%d, %d, %d, false>" % (tile, kt, act)
    return {"project": "k_project<3>", "sh_bwd": "k_sh_bwd<3>"}.get(kind, "k_" + kind)


def measured_traffic(kernel):
    """HBM bytes per dispatch of one kernel (its exact profiled name) from a
    committed rocprofv3 summary under profiles/, if that summary was taken on
    the current HIP sources."""
    import glob
    import re as _re
    from paper_2412_04459_amd.profsum import source_hash
    h = source_hash()
    for f in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        m = _re.search(r"```json\n(.*?)\n```", open(f).read(), _re.S)
        if not m:
            continue
        blk = json.loads(m.group(1))
        if blk.get("source_hash") != h:
            continue
        for k, v in blk.get("traffic", {}).items():
            if k == kernel and blk.get("fetch_factor"):
                return v["bytes_scaled"], os.path.relpath(f, ROOT)
    return None, None


def measured_counters(kernel):
    """Hardware counters per dispatch of one kernel (mean over its dispatches)
    from a committed rocprofv3 --pmc summary under profiles/ taken on the
    current HIP sources: {counter: value}, and the summary's path."""
    import glob
    import re as _re
    from paper_2412_04459_amd.profsum import source_hash
    h = source_hash()
    out, src = {}, None
    for f in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        m = _re.search(r"```json\n(.*?)\n```", open(f).read(), _re.S)
        if not m:
            continue
        blk = json.loads(m.group(1))
        if blk.get("source_hash") != h:
            continue
        c = blk.get("counters", {}).get(kernel)
        if c:
            out.update(c)
            src = os.path.relpath(f, ROOT)
    return out, src


def atomic_probe_run(n_rows, log, n_waves=1 << 18, iters=32, reps=5):
    """Float atomic adds in the render backward's flush pattern (11 lanes per
    instruction over a voxel's corner and colour rows, no return) on an array
    of n_rows voxels: instructions and lane atomics per second, timed with
    HIP events on the launch stream."""
    import ctypes
    import torch
    from paper_2412_04459_amd import _abi
    corner = torch.zeros((n_rows, 8), dtype=torch.float32, device="cuda")
    colour = torch.zeros((n_rows, 3), dtype=torch.float32, device="cuda")
    st = torch.cuda.current_stream()
    sp = ctypes.c_void_p(st.cuda_stream)

    def launch():
        rc = _abi.svr_atomic_probe(ctypes.c_void_p(corner.data_ptr()),
                                   ctypes.c_void_p(colour.data_ptr()), n_rows, n_waves, iters, sp)
        _abi.check(rc, "svr_atomic_probe")

    launch()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        launch()
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    total = float(corner.double().sum().item() + colour.double().sum().item())
    expect = 11.0 * n_waves * iters * (reps + 1)
    assert total == expect, "atomic probe lost updates: %r vs %r" % (total, expect)
    inst = n_waves * iters
    log("atomic probe: %d instructions (11 lanes) over %d voxels in %.3f ms" % (inst, n_rows, ms))
    del corner, colour
    return {"pattern": "11-lane float atomic add, no return, random voxel rows (8 + 3 floats)",
            "rows": n_rows, "instructions": inst, "ms": ms,
            "instructions_per_s": inst / (ms / 1e3), "lane_atomics_per_s": 11 * inst / (ms / 1e3)}


def small_configs_run(log, no_cpu, cpu_seconds):
    """The two small workloads: a plain forward render of the ~3.3k-voxel
    level-6 sphere shell at 64x64 (K = 1, SH degree 0) and fwd+bwd of the
    ~184k-voxel spheres-and-plane scene at 800x800 (K = 1, SH degree 3), each
    timed on the GPU (eager launches, median of repeated frames) and, unless
    no_cpu, the oracle on the host (all threads; cfg0 full frame, the other on
    a pixel sample)."""
    import torch
    from paper_2412_04459_amd import scenes as S
    from paper_2412_04459_amd.render import DeviceScene, Rasterizer
    out = {}
    from paper_2412_04459_amd.render import zcurve_relabel
    for name, bwd in (("sphere_shell_3k", False), ("spheres_plane_184k", True)):
        wl = S.workload(name)
        scene, _ = zcurve_relabel(wl.scene)
        cam = wl.cameras[0]
        P = cam.W * cam.H
        ds = DeviceScene(scene)
        probe = Rasterizer(ds, [cam], K=wl.K, sync_count=True, tile=8)
        probe.preprocess()
        cap = int(probe.n_entries * 1.1) + 4096
        del probe
        r = Rasterizer(ds, [cam], K=wl.K, capacity=cap, sync_count=False, tile=8)
        g = torch.from_numpy(S.upstream_grads(P, wl.grad_seed)).cuda()
        rgba = torch.empty((P, 4), dtype=torch.float32, device="cuda")
        gg = torch.empty(ds.n_grid, dtype=torch.float32, device="cuda")
        gs = torch.empty_like(ds.sh)
        # the frame as one captured hipGraph (small frames are launch-bound)
        r.capture(rgba, g if bwd else None, gg if bwd else None, gs if bwd else None)

        def frame():
            r.replay()

        for _ in range(3):
            frame()
        torch.cuda.synchronize()
        times = []
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        for _ in range(15):
            e0.record()
            for _ in range(4):
                frame()
            e1.record()
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1) / 4)
        ms = float(np.median(times))
        assert r.check_overflow() <= cap
        r.release_graph()
        row = {"workload": "%s, %dx%d, K=%d, %s, one hipGraph per frame" % (
                   name, cam.W, cam.H, wl.K, "fwd+bwd" if bwd else "forward only"),
               "n_voxels": scene.n_voxels, "ms_per_frame": ms,
               "mpix_s": P / (ms / 1e3) / 1e6, "frames_per_s": 1e3 / ms}
        if not no_cpu:
            import oracle
            threads = len(os.sched_getaffinity(0))
            if bwd:
                row["cpu_baseline"] = cpu_baseline(scene, cam, wl.K, cpu_seconds / 3)
            else:
                t0 = time.perf_counter()
                oracle.render(scene, cam, K=wl.K, nthreads=threads)
                dt = time.perf_counter() - t0
                row["cpu_baseline"] = {"value": P / dt / 1e6, "unit": "Mpix/s", "cores": threads,
                                       "kind": "oracle", "sample": "full frame, FP64 forward"}
        log("%s: %.3f ms per frame (%.0f Mpix/s)" % (name, ms, P / (ms / 1e3) / 1e6))
        out[name] = row
        del r, ds, rgba, g, gg, gs
        torch.cuda.empty_cache()
    return out


def supersampled_run(ds, cams, K, tile, grad, steps, log):
    """Anti-aliased frames (Sec. 3.1.2): each view rendered at ss times its
    resolution, downsampled by the tent filter with a background colour, and
    differentiated through both; ms per frame and target Mpix/s."""
    import torch
    from paper_2412_04459_amd.render import Rasterizer, downsample, supersampled_camera
    out = {}
    W, H = cams[0].W, cams[0].H
    bg = [0.5, 0.5, 0.5]
    for ss in (1.1, 1.5):
        hi = [supersampled_camera(c, ss) for c in cams]
        probe = Rasterizer(ds, [hi[0]], K=K, sync_count=True, tile=tile)
        e_max = 0
        for c in hi[:8]:
            probe.set_cameras([c])
            probe.preprocess()
            e_max = max(e_max, probe.n_entries)
        del probe
        r = Rasterizer(ds, [hi[0]], K=K, capacity=int(e_max * 1.2) + 4096, sync_count=False,
                       tile=tile)
        Wh, Hh = hi[0].W, hi[0].H
        rgba = torch.empty((Wh * Hh, 4), dtype=torch.float32, device="cuda")
        lo = torch.empty((W * H, 4), dtype=torch.float32, device="cuda")
        from paper_2412_04459_amd import _abi
        from paper_2412_04459_amd.render import _bg_arr, _ptr, _stream
        g_hi = torch.empty_like(rgba)
        bga = _bg_arr(bg)

        def step(i):
            r.set_cameras([hi[i % len(hi)]])
            r.forward(out=rgba)
            _abi.svr_downsample(_ptr(rgba), Wh, Hh, _ptr(lo), W, H, bga, _stream())
            _abi.svr_downsample_bwd(_ptr(grad), W, H, _ptr(g_hi), Wh, Hh, bga, _stream())
            r.backward(g_hi)

        for i in range(3):
            step(i)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for i in range(steps):
            step(i)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        over = r.check_overflow()
        out["ss%.1f" % ss] = {"render_resolution": "%dx%d" % (Wh, Hh), "ms_per_frame": ms,
                              "target_mpix_s": W * H / (ms / 1e3) / 1e6,
                              "overflow": over > r.capacity}
        log("supersampled ss=%.1f (%dx%d): %.3f ms per fwd+bwd frame" % (ss, Wh, Hh, ms))
        del r, rgba, lo, g_hi
        torch.cuda.empty_cache()
    return out


def mesh_run(cams, K, tile, reps, log):
    """Mesh extraction (Sec. 3.2.4) on the opaque variant of the orbit scene
    (same octree, surfaces opaque, as meshing assumes): the views' rgba and
    depth rendered, then TSDF fusion of all views at the grid points and
    marching cubes over the voxels at iso 0, each timed on its own; ms per
    call and HBM rates from
    the algorithmic bytes (TSDF: 12 B position + 8 B outputs per grid point
    and 8 B depth + opacity per accepted observation; marching cubes: 48 B
    of voxel record + 8 B field and weight per grid point + 60 B per
    triangle)."""
    import torch
    from paper_2412_04459_amd import scenes as S
    from paper_2412_04459_amd.render import (DeviceScene, Rasterizer, marching_cubes,
                                             marching_cubes_into, morton_order, tsdf_fuse)
    scene = S.spheres_background_scene(opaque=True)
    ds = DeviceScene(scene)
    rast = Rasterizer(ds, [cams[0]], K=K, tile=tile)
    P = sum(c.W * c.H for c in cams)
    rgba = torch.empty((P, 4), dtype=torch.float32, device="cuda")
    dep = torch.empty(P, dtype=torch.float32, device="cuda")
    off = 0
    for c in cams:
        n = c.W * c.H
        rast.set_cameras([c])
        rast.forward(out=rgba[off:off + n], depth=dep[off:off + n])
        off += n
    torch.cuda.synchronize()
    trunc = 4.0 * scene.world_size / 2 ** scene.max_level
    # Z-curve visit orders of the grid points and voxels (once per scene)
    g_order = morton_order(ds.grid_pos, ds.world_lo, ds.world_size)
    v_order = morton_order(ds.center, ds.world_lo, ds.world_size)
    tsdf, w = tsdf_fuse(ds.grid_pos, cams, dep, trunc, rgba, 0.5, order=g_order)
    keys, pos = marching_cubes(ds, tsdf, 0.0, w, order=v_order)
    n_tri = keys.shape[0]
    cap = n_tri + 1024
    keys = torch.empty((cap, 3, 2), dtype=torch.int32, device="cuda")
    pos = torch.empty((cap, 3, 3), dtype=torch.float32, device="cuda")
    count = torch.zeros(1, dtype=torch.int64, device="cuda")
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    t_ms = timed(lambda: tsdf_fuse(ds.grid_pos, cams, dep, trunc, rgba, 0.5, tsdf, w,
                                   order=g_order))
    m_ms = timed(lambda: marching_cubes_into(ds, tsdf, keys, pos, count, 0.0, w, order=v_order))
    t_ms_own = timed(lambda: tsdf_fuse(ds.grid_pos, cams, dep, trunc, rgba, 0.5, tsdf, w))
    m_ms_own = timed(lambda: marching_cubes_into(ds, tsdf, keys, pos, count, 0.0, w))
    assert int(count.item()) == n_tri
    M, N = scene.n_grid, scene.n_voxels
    obs = float(w.double().sum().item())
    t_bytes = 20.0 * M + 8.0 * obs
    m_bytes = 48.0 * N + 8.0 * M + 60.0 * n_tri
    observed = int((w > 0).sum().item())
    log("mesh: tsdf %.3f ms (%d views, %d grid points), marching cubes %.3f ms, %d triangles "
        "(own order: %.3f / %.3f ms)" % (t_ms, len(cams), M, m_ms, n_tri, t_ms_own, m_ms_own))
    del rast, ds
    return {"scene": "orbit scene, opaque surfaces", "views": len(cams), "grid_points": M,
            "voxels": N, "trunc": trunc,
            "observed_grid_points": observed, "triangles": n_tri,
            "visit_order": "Z-curve of grid points / voxel centres (svr_morton_keys)",
            "tsdf_ms_own_order": t_ms_own, "marching_cubes_ms_own_order": m_ms_own,
            "tsdf": {"ms": t_ms, "bytes": t_bytes, "achieved_GBs": t_bytes / t_ms / 1e6,
                     "frac": t_bytes / t_ms / 1e6 / HBM_PEAK_GBS},
            "marching_cubes": {"ms": m_ms, "bytes": m_bytes, "achieved_GBs": m_bytes / m_ms / 1e6,
                               "frac": m_bytes / m_ms / 1e6 / HBM_PEAK_GBS}}


def large_scene_run(log):
    """~8M voxels (max level 14), 16 views at 1920x1080, K = 1, fwd+bwd of all
    16 views in one batched graph (16x16 tiles, one launch per stage), plus
    the memory footprint of the duplicated list and of the sort."""
    import torch
    from paper_2412_04459_amd import scenes as S
    from paper_2412_04459_amd.autotune import time_batch
    from paper_2412_04459_amd.render import BatchRenderer, DeviceScene, Rasterizer

    from paper_2412_04459_amd.render import zcurve_relabel
    t0 = time.time()
    scene, _ = zcurve_relabel(S.large_shells_scene())
    cams = S.orbit_cameras_1080p()
    log("large scene: %d voxels, %d grid points (%.0fs)" % (scene.n_voxels, scene.n_grid,
                                                          time.time() - t0))
    ds = DeviceScene(scene)
    del scene
    P = sum(c.W * c.H for c in cams)
    grad = torch.from_numpy(S.upstream_grads(P, 4)).cuda()
    out = {"n_voxels": ds.n_voxels, "views": len(cams), "resolution": "1920x1080", "K": 1}
    for tile in (8, 16):
        br = BatchRenderer(ds, cams, 1, group=len(cams), tile=tile, persistent=0)
        br.capture(grad)
        ms = time_batch(br, reps=3)
        r = br.rasts[0]
        E = r.check_overflow()
        out["tile%d" % tile] = {
            "ms": ms, "mpix_s": P / (ms / 1e3) / 1e6, "frames_per_s": len(cams) / (ms / 1e3),
            "entries": E, "entries_per_view": E / len(cams),
            "list_bytes_at_E": 2 * E * 12,            # keys + values, double buffered
            "workspace_bytes": br.workspace_bytes(), "workspace_parts": br.workspace_parts(),
            "scene_bytes": ds.nbytes(), "overflow": E > r.capacity}
        log("large scene, tile %d: %.1f ms for 16 views (%.0f Mpix/s), E = %d, workspace %.2f GB"
            % (tile, ms, P / (ms / 1e3) / 1e6, E, br.workspace_bytes() / 1e9))
        del br
        torch.cuda.empty_cache()
    return out


def batched_comparison(ds, K, log):
    """24 cameras of uneven resolution over the same scene: 24 single-view
    frames (one fwd+bwd each, eager launches) against the autotuned batched
    path (camera groups in one launch per stage, each group one hipGraph)."""
    import torch
    from paper_2412_04459_amd import scenes as S
    from paper_2412_04459_amd.autotune import time_batch, tune
    from paper_2412_04459_amd.render import BatchRenderer, Rasterizer

    cams = S.mixed_resolution_cameras()
    P = sum(c.W * c.H for c in cams)
    grad = torch.from_numpy(S.upstream_grads(P, 3)).cuda()
    # single-view launches
    singles = []
    off = 0
    for c in cams:
        probe = Rasterizer(ds, [c], K=K, sync_count=True)
        probe.preprocess()
        cap = int(probe.n_entries * 1.1) + 4096
        del probe
        r = Rasterizer(ds, [c], K=K, capacity=cap, sync_count=False)
        singles.append((r, grad[off:off + c.W * c.H]))
        off += c.W * c.H

    def run_singles():
        for r, g in singles:
            r.forward()
            r.backward(g)

    run_singles()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    reps = 3
    e0.record()
    for _ in range(reps):
        run_singles()
    e1.record()
    torch.cuda.synchronize()
    single_ms = e0.elapsed_time(e1) / reps
    del singles
    torch.cuda.empty_cache()
    log("24 single-view frames: %.2f ms" % single_ms)
    res = tune(ds, cams, K, grad, reps=3, log=log)
    br = BatchRenderer(ds, cams, K, group=res["group"], tile=res["tile"],
                       persistent=res["persistent"])
    br.capture(grad)
    batched_ms = time_batch(br, reps=5)
    ok = br.check_overflow()
    ws = br.workspace_bytes()
    del br
    torch.cuda.empty_cache()
    res_rows = [{k: r[k] for k in ("group", "tile", "persistent", "ms")} for r in res["table"]]
    return {"cameras": len(cams), "pixels": P,
            "resolutions": sorted({"%dx%d" % (c.W, c.H) for c in cams}),
            "single_view_ms": single_ms, "single_view_mpix_s": P / (single_ms / 1e3) / 1e6,
            "batched_ms": batched_ms, "batched_mpix_s": P / (batched_ms / 1e3) / 1e6,
            "speedup": single_ms / batched_ms, "overflow": not ok,
            "autotuned": {"tile": res["tile"], "persistent": res["persistent"],
                          "cameras_per_launch": res["group"]},
            "workspace_bytes": ws, "autotune_table": res_rows}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=72)
    ap.add_argument("--warmup", type=int, default=8)
    ap.add_argument("--views", type=int, default=36)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--main-only", action="store_true",
                    help="time only the headline frames (profiled runs: every launch of the "
                         "headline kernels then belongs to the headline workload)")
    ap.add_argument("--mesh-only", action="store_true",
                    help="run only the mesh extraction (TSDF fusion + marching cubes) timing and "
                         "print its JSON object")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--tile", type=int, default=0, choices=(0, 8, 16, 32),
                    help="tile edge of the headline frames (0: the fastest of 8, 16 and 32 by a "
                         "short measurement)")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the 24-camera batched comparison")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the ~8M-voxel scene (16 views at 1920x1080, batched)")
    ap.add_argument("--no-small", action="store_true",
                    help="skip the two small workloads (3.3k voxels at 64x64, 184k at 800x800)")
    ap.add_argument("--calibrate", action="store_true",
                    help="run a plain 1 GiB device copy first (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: every box in this setup has a single MI355X, "
              "and multi-GPU sharding is a design note, not a measured path.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2412_04459_amd import _abi
    from paper_2412_04459_amd import scenes as S
    from paper_2412_04459_amd.render import DeviceScene, Rasterizer, zcurve_relabel

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.calibrate:
        # a plain copy of known size, for scaling FETCH_SIZE / WRITE_SIZE
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.mesh_only:
        cams = S.orbit_cameras_1297x840(n=args.views)
        print(json.dumps({"mesh": mesh_run(cams, 2, 8, args.steps, log)}), flush=True)
        return
    t0 = time.time()
    # voxels stored in octree-path order (relabeled once at load; the
    # generator's shuffled order stands for an arbitrary caller order)
    scene, _ = zcurve_relabel(S.spheres_background_scene())
    cams = S.orbit_cameras_1297x840(n=args.views)
    K = 2
    log("scene: %d voxels, %d grid points (%.1fs)" % (scene.n_voxels, scene.n_grid, time.time() - t0))
    ds = DeviceScene(scene)
    P = cams[0].W * cams[0].H
    S_floats = 3 * (scene.sh_degree + 1) ** 2

    # capacity from one counted pass over the orbit
    probe = Rasterizer(ds, [cams[0]], K=K, sync_count=True)
    e_max = 0
    for c in cams:
        probe.set_cameras([c])
        probe.preprocess()
        e_max = max(e_max, probe.n_entries)
    del probe
    cap = int(e_max * 1.1) + 4096
    grad = torch.from_numpy(S.upstream_grads(P, 2)).cuda()
    # tile edge: a short measurement over the orbit picks it (as the autotuner
    # does for batches); the capacity above covers 16x16 tiles, so the other
    # edges get their own counted pass
    tile_ms = {}
    for tile in ((8, 16, 32) if args.tile == 0 else (args.tile,)):
        probe = Rasterizer(ds, [cams[0]], K=K, sync_count=True, tile=tile)
        e_t = 0
        for c in cams[:: max(1, len(cams) // 6)]:
            probe.set_cameras([c])
            probe.preprocess()
            e_t = max(e_t, probe.n_entries)
        del probe
        r = Rasterizer(ds, [cams[0]], K=K, capacity=int(e_t * 1.25) + 4096, sync_count=False,
                       tile=tile)
        for i in range(2):
            r.set_cameras([cams[i]])
            r.forward()
            r.backward(grad)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for i in range(6):
            r.set_cameras([cams[(5 * i) % len(cams)]])
            r.forward()
            r.backward(grad)
        e1.record()
        torch.cuda.synchronize()
        tile_ms[tile] = e0.elapsed_time(e1) / 6
        del r
    tile = min(tile_ms, key=tile_ms.get)
    log("tile edge: %s -> %d" % (", ".join("%d: %.3f ms" % kv for kv in sorted(tile_ms.items())),
                                  tile))
    probe = Rasterizer(ds, [cams[0]], K=K, sync_count=True, tile=tile)
    e_max = 0
    for c in cams:
        probe.set_cameras([c])
        probe.preprocess()
        e_max = max(e_max, probe.n_entries)
    del probe
    cap = int(e_max * 1.1) + 4096
    rast = Rasterizer(ds, [cams[0]], K=K, capacity=cap, sync_count=False, tile=tile)

    # per-view statistics (untimed)
    stats = []
    for c in cams:
        rast.set_cameras([c])
        rast.preprocess()
        rast.sort()
        stats.append(rast.stats())
    st = np.array(stats, dtype=np.float64)  # E, walked pairs, tests, hits, in-view voxels
    E_mean, pairs_mean, tests_mean, hits_mean, Nv_mean = st.mean(0)
    log("mean per view: E=%.0f pairs=%.3g tests=%.3g hits=%.3g in-view voxels=%.0f" % (
        E_mean, pairs_mean, tests_mean, hits_mean, Nv_mean))

    def step(i):
        rast.set_cameras([cams[i % len(cams)]])
        rast.forward()
        rast.backward(grad)

    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    _abi.svr_timing_enable(1)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    for i in range(args.steps):
        step(i)
    ev1.record()
    torch.cuda.synchronize()
    elapsed_ms = ev0.elapsed_time(ev1)
    ktimes = _abi.kernel_times()
    _abi.svr_timing_enable(0)
    over = rast.check_overflow()
    assert over <= cap, "entry capacity overflow during the timed region"
    # same workload without per-kernel events, for the headline number
    torch.cuda.synchronize()
    ev0.record()
    for i in range(args.steps):
        step(i)
    ev1.record()
    torch.cuda.synchronize()
    elapsed_ms = min(elapsed_ms, ev0.elapsed_time(ev1))
    eager_ms_step = elapsed_ms / args.steps

    def optional_timings():
        """The same steps with the training statistics on (max blending weight
        in the forward, subdivision priority in the backward), then rendering
        and differentiating depth and normal images too; ms per step each."""
        mw = torch.zeros(scene.n_voxels, dtype=torch.float32, device="cuda")
        pr = torch.zeros_like(mw)

        def step_stats(i):
            rast.set_cameras([cams[i % len(cams)]])
            rast.forward(max_weight=mw)
            rast.backward(grad, priority=pr)

        torch.cuda.synchronize()
        ev0.record()
        for i in range(args.steps):
            step_stats(i)
        ev1.record()
        torch.cuda.synchronize()
        stats_ms_step = ev0.elapsed_time(ev1) / args.steps
        del mw, pr

        # the same steps rendering and differentiating depth and normal images too
        dep = torch.empty(P, dtype=torch.float32, device="cuda")
        nrm = torch.empty((P, 3), dtype=torch.float32, device="cuda")
        gdep = torch.from_numpy(np.random.default_rng(3).normal(size=P).astype(np.float32)).cuda()
        gnrm = torch.from_numpy(np.random.default_rng(4).normal(size=(P, 3)).astype(np.float32)).cuda()

        def step_aux(i):
            rast.set_cameras([cams[i % len(cams)]])
            rast.forward(depth=dep, normal=nrm)
            rast.backward(grad, grad_depth=gdep, grad_normal=gnrm)

        for i in range(2):
            step_aux(i)
        torch.cuda.synchronize()
        ev0.record()
        for i in range(args.steps):
            step_aux(i)
        ev1.record()
        torch.cuda.synchronize()
        aux_ms_step = ev0.elapsed_time(ev1) / args.steps
        del dep, nrm, gdep, gnrm

        # the same steps through torch.autograd.Function (render(), then
        # backward of the rgba with the same upstream gradient): the GPU work
        # is the eager step's, the difference is the autograd host path
        from paper_2412_04459_amd.render import render as svr_render_fn
        gp = ds.grid_raw.detach().clone().requires_grad_(True)
        sp = ds.sh.detach().clone().requires_grad_(True)

        def step_ag(i):
            rast.set_cameras([cams[i % len(cams)]])
            rgba = svr_render_fn(rast, gp, sp)
            rgba.backward(grad)
            gp.grad = None
            sp.grad = None

        for i in range(2):
            step_ag(i)
        torch.cuda.synchronize()
        ev0.record()
        for i in range(args.steps):
            step_ag(i)
        ev1.record()
        torch.cuda.synchronize()
        ag_ms_step = ev0.elapsed_time(ev1) / args.steps
        del gp, sp

        return stats_ms_step, aux_ms_step, ag_ms_step

    stats_ms_step, aux_ms_step, ag_ms_step = (None, None, None) if args.main_only else optional_timings()

    # the same frames replayed from one captured hipGraph per view (no host
    # launch overhead); this is the headline number
    gstream = torch.cuda.Stream()
    g_rgba = torch.empty((P, 4), dtype=torch.float32, device="cuda")
    g_grid = torch.empty(scene.n_grid, dtype=torch.float32, device="cuda")
    g_sh = torch.empty_like(ds.sh)
    n_graphs = rast.capture_views(cams, g_rgba, grad, g_grid, g_sh, gstream)
    for i in range(args.warmup):
        rast.replay_view(i % n_graphs, gstream)
    torch.cuda.synchronize()
    ev0.record(gstream)
    for i in range(args.steps):
        rast.replay_view(i % n_graphs, gstream)
    ev1.record(gstream)
    torch.cuda.synchronize()
    elapsed_ms = ev0.elapsed_time(ev1)
    over = rast.check_overflow()
    assert over <= cap, "entry capacity overflow during the graph replays"
    rast.release_graph()

    # the headline takes the faster of the two launch modes of the same
    # steps (the per-view graph replays, the eager launches); both are kept
    graph_ms_step = elapsed_ms / args.steps
    ms_step = min(graph_ms_step, eager_ms_step)
    launch = ("one hipGraph per view, replayed on one stream" if graph_ms_step <= eager_ms_step
              else "eager launches on one stream (faster than the per-view hipGraph replays here)")
    mpix = P / (ms_step / 1e3) / 1e6
    per_kernel = {k: {"ms_per_step": v[0] / args.steps, "launches_per_step": v[1] / args.steps,
                      "avg_us": 1e3 * v[0] / max(v[1], 1)} for k, v in ktimes.items()}
    dom = max(ktimes, key=lambda k: ktimes[k][0])
    dom_avg_s = ktimes[dom][0] / 1e3 / ktimes[dom][1]
    if dom in ("render_fwd", "render_bwd"):
        hk = "hit_fwd" if dom == "render_fwd" else "hit_bwd"
        counts = {}
        for nm, c in OPS.items():
            o = pairs_mean * c["pair"] + hits_mean * c[hk](K)
            counts[nm] = {"per_pair": c["pair"], "per_hit": c[hk](K), "ops_per_launch": o,
                          "achieved": o / dom_avg_s / 1e12,
                          "frac": o / dom_avg_s / 1e12 / VALU_PEAK_TOPS}
        ops = counts["design"]["ops_per_launch"]
        ach = ops / dom_avg_s / 1e12
        roof = {"kernel": dom, "bound": "alu", "achieved": ach, "peak": VALU_PEAK_TOPS,
                "unit": "Tops/s", "frac": ach / VALU_PEAK_TOPS, "traffic": None,
                "ops_per_launch": ops, "op_counts": counts,
                "units_per_launch": {"pairs": pairs_mean, "hits": hits_mean}}
    else:
        b = kernel_bytes(dom, scene.n_voxels, Nv_mean, E_mean, P, S_floats, None)
        ach = b / dom_avg_s / 1e9
        roof = {"kernel": dom, "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": ach / HBM_PEAK_GBS, "traffic": None,
                "bytes_per_launch": b}
    roof["symbol"] = kernel_symbol(dom, tile, K)
    tb, tsrc = measured_traffic(roof["symbol"])
    if tb is not None:
        roof["traffic"] = tb
        roof["traffic_source"] = tsrc
    # counter evidence for the render kernels: VALU issue (VALUBusy: share of
    # time the SIMDs issue VALU) and lane occupancy (VALUUtilization: active
    # lanes per issued VALU instruction), LDS, waits and atomics
    counters = {}
    for kind in ("render_fwd", "render_bwd"):
        sym = kernel_symbol(kind, tile, K)
        c, csrc = measured_counters(sym)
        if c:
            counters[kind] = {"symbol": sym, "source": csrc, **c}
    if counters:
        roof["counters"] = counters
    probe = atomic_probe_run(scene.n_voxels, log)
    c_probe, _ = measured_counters("k_atomic_probe")
    atomics = {"probe": probe}
    bw = counters.get("render_bwd", {})
    if bw.get("TCP_TCC_ATOMIC_WITHOUT_RET_REQ_sum") and c_probe.get("TCP_TCC_ATOMIC_WITHOUT_RET_REQ_sum"):
        # requests to L2 per second: the backward (its profiled requests per
        # dispatch over its live duration) against the probe (requests per
        # dispatch of the same profile over the probe's live duration)
        rb = bw["TCP_TCC_ATOMIC_WITHOUT_RET_REQ_sum"] / (ktimes["render_bwd"][0] / 1e3 / ktimes["render_bwd"][1])
        rp = c_probe["TCP_TCC_ATOMIC_WITHOUT_RET_REQ_sum"] / (probe["ms"] / 1e3)
        atomics["render_bwd"] = {"l2_atomic_requests_per_launch": bw["TCP_TCC_ATOMIC_WITHOUT_RET_REQ_sum"],
                                 "requests_per_s": rb, "probe_requests_per_s": rp, "frac": rb / rp,
                                 "source": bw.get("source")}
    fb = frame_bytes(scene.n_voxels, Nv_mean, E_mean, P, S_floats)
    fbytes = sum(fb.values())
    frame_gbs = fbytes / (ms_step / 1e3) / 1e9
    out = {
        "metric": METRIC,
        "value": mpix,
        "unit": "Mpix/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32",
        "data": "synthetic",
        "config": {"workload": "fwd+bwd, %d voxels (max level 12, SH degree 3), %dx%d, K=%d, "
                               "explin, %d-view seeded orbit" % (scene.n_voxels, cams[0].W,
                                                                 cams[0].H, K, len(cams)),
                   "n_voxels": scene.n_voxels, "pixels": P, "entries_mean": E_mean, "tile": tile,
                   "tile_ms": tile_ms,
                   "in_view_voxels_mean": Nv_mean, "hits_per_pixel": hits_mean / P},
        "frames_per_s": 1e3 / ms_step,
        "launch": launch,
        "graph": {"ms_per_step": graph_ms_step, "mpix_s": P / (graph_ms_step / 1e3) / 1e6},
        "eager": {"ms_per_step": eager_ms_step, "mpix_s": P / (eager_ms_step / 1e3) / 1e6},
        "with_train_stats": None if stats_ms_step is None else {
            "ms_per_step": stats_ms_step, "overhead": stats_ms_step / eager_ms_step - 1.0},
        "with_depth_normal": None if aux_ms_step is None else {
            "ms_per_step": aux_ms_step, "overhead": aux_ms_step / eager_ms_step - 1.0},
        "autograd": None if ag_ms_step is None else {
            "ms_per_step": ag_ms_step, "overhead": ag_ms_step / eager_ms_step - 1.0,
            "path": "torch.autograd.Function (render(), rgba.backward), eager launches"},
        "frame_hbm": {"bytes": fbytes, "achieved_GBs": frame_gbs, "peak_GBs": HBM_PEAK_GBS,
                      "frac": frame_gbs / HBM_PEAK_GBS},
        "roofline": roof,
        "atomics": atomics,
        "kernels": per_kernel,
        "stages": stage_rows(per_kernel, scene.n_voxels, Nv_mean, E_mean, P, S_floats),
        "paper_context": PAPER_CONTEXT,
    }
    if not args.main_only:
        out["supersampled"] = supersampled_run(ds, cams, K, tile, grad, min(args.steps, 24), log)
        out["mesh"] = mesh_run(cams, K, tile, 20, log)
    if not (args.no_batched or args.main_only):
        out["batched"] = batched_comparison(ds, K, log)
    if not (args.no_small or args.main_only):
        out["small_configs"] = small_configs_run(log, args.no_cpu, args.cpu_seconds)
    if not (args.no_large or args.main_only):
        del rast
        torch.cuda.empty_cache()
        out["large"] = large_scene_run(log)
    if not (args.no_cpu or args.main_only):
        log("timing the oracle on the host ...")
        out["cpu_baseline"] = cpu_baseline(scene, cams[0], K, args.cpu_seconds)
        one = cpu_baseline(scene, cams[0], K, args.cpu_seconds / 2, threads=1)
        out["cpu_baseline"]["single_thread"] = {k: one[k] for k in ("value", "cores", "sample")}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
