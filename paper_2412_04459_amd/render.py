"""Torch-facing wrapper of the C ABI: device-resident scene, a rasterizer that
owns its workspace, and a ``torch.autograd.Function``.

PyTorch supplies device memory and the stream only; each stage is one call
into ``libsvraster.so``.  There is no CPU or PyTorch fallback: without a GPU
and the built library every entry point raises.
"""
from __future__ import annotations

import ctypes
import dataclasses
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import _abi
from ._abi import check


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _extra(**tensors):
    """svr_extra for the given tensors (float32, contiguous; None: off), or
    None when all are None."""
    if all(t is None for t in tensors.values()):
        return None
    ex = _abi.svr_extra()
    for name, t in tensors.items():
        if t is None:
            continue
        if t.dtype != torch.float32 or not t.is_contiguous():
            raise ValueError("%s must be a contiguous float32 tensor" % name)
        setattr(ex, name, t.data_ptr())
    return ex


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def grid_zcurve_order(scene) -> np.ndarray:
    """Permutation of the grid points along the Z-curve of their integer
    positions at the finest level (x, y, z bits interleaved from the top, x
    first, as in the octree path's child index 4x + 2y + z)."""
    L = int(scene.max_level)
    lo = np.asarray(scene.world_center, np.float64) - 0.5 * float(scene.world_size)
    step = float(scene.world_size) / float(1 << L)
    g = np.rint((np.asarray(scene.grid_pos, np.float64) - lo[None, :]) / step).astype(np.uint64)
    code = np.zeros(g.shape[0], np.uint64)
    for b in range(L, -1, -1):
        for a in range(3):
            code = (code << np.uint64(1)) | ((g[:, a] >> np.uint64(b)) & np.uint64(1))
    return np.argsort(code, kind="stable")


def zcurve_relabel(scene, grid_points: bool = True):
    """The scene with its voxels stored in octree-path order (a depth-first,
    Z-curve walk of the leaves) and, with ``grid_points``, its grid points
    stored along the same curve; and the voxel permutation: stored voxel i is
    voxel order[i] of the given scene.  Only labels change (geometry and
    parameters are the same), so every output is the given scene's,
    relabeled.  Neighbouring voxels and grid points then sit near each other
    in memory: the corner gathers of the projection and of the grid gradient
    hit the same cache lines, and a tile's entries (sorted in a Z-curve
    order) read neighbouring records."""
    order = np.argsort(np.asarray(scene.octpath, np.uint64), kind="stable")
    out = scene.subset(order)
    if grid_points:
        gorder = grid_zcurve_order(out)
        inv = np.empty_like(gorder)
        inv[gorder] = np.arange(gorder.shape[0], dtype=gorder.dtype)
        out = dataclasses.replace(
            out, vox_grid=np.ascontiguousarray(inv[out.vox_grid].astype(np.int32)),
            grid_pos=np.ascontiguousarray(out.grid_pos[gorder]),
            grid_raw=np.ascontiguousarray(out.grid_raw[gorder]))
    return out, order


class DeviceScene:
    """Scene arrays resident in device memory (layouts as in svr_scene), in
    the voxel order given (zcurve_relabel gives the order the benchmark
    stores)."""

    def __init__(self, scene, device="cuda", grid_adjacency: bool = True,
                 order_ranks: bool = True):
        if not torch.cuda.is_available():
            raise RuntimeError("DeviceScene needs a HIP device")
        dev = torch.device(device)
        self.n_voxels = int(scene.n_voxels)
        self.n_grid = int(scene.n_grid)
        # bounding cube of the scene (visit orders of the mesh kernels)
        self.world_lo = [float(x) - 0.5 * float(scene.world_size) for x in scene.world_center]
        self.world_size = float(scene.world_size)
        self.sh_degree = int(scene.sh_degree)
        self.max_level = int(scene.max_level)
        self.center = torch.from_numpy(np.ascontiguousarray(scene.center, np.float32)).to(dev)
        self.size = torch.from_numpy(np.ascontiguousarray(scene.size, np.float32)).to(dev)
        self.octpath = torch.from_numpy(
            np.ascontiguousarray(scene.octpath, np.uint64).view(np.int64)).to(dev)
        self.vox_grid = torch.from_numpy(np.ascontiguousarray(scene.vox_grid, np.int32)).to(dev)
        self.grid_raw = torch.from_numpy(np.ascontiguousarray(scene.grid_raw, np.float32)).to(dev)
        self.sh = torch.from_numpy(np.ascontiguousarray(scene.sh, np.float32)).to(dev)
        self.device = self.grid_raw.device
        gp = getattr(scene, "grid_pos", None)
        self.grid_pos = None if gp is None else torch.from_numpy(
            np.ascontiguousarray(np.asarray(gp, np.float32).T)).to(dev)  # [3][M]
        self.adj_off = self.adj = None
        if grid_adjacency:
            self.build_adjacency()
        self.rank = None
        if order_ranks:
            self.build_order_ranks()

    def build_order_ranks(self):
        """Order ranks of the (voxel, sign) pairs (svr_build_order_ranks): the
        per-frame sort key then needs ceil(log2(8N)) bits below the tile id
        instead of 3 max_level + 3."""
        rank = torch.empty(max(1, 8 * self.n_voxels), dtype=torch.int32, device=self.device)
        nb = _abi.svr_order_rank_scratch_bytes(self.n_voxels, self.max_level)
        scratch = torch.empty(nb + 256, dtype=torch.uint8, device=self.device)
        p = (scratch.data_ptr() + 255) // 256 * 256
        check(_abi.svr_build_order_ranks(_ptr(self.octpath), self.n_voxels, self.max_level,
                                         _ptr(rank), ctypes.c_void_p(p), nb, _stream()),
              "svr_build_order_ranks")
        torch.cuda.current_stream().synchronize()
        del scratch
        self.rank = rank

    def build_adjacency(self):
        """Corner adjacency of the grid points (svr_build_grid_adjacency): makes the
        grid gradient a deterministic gather instead of atomics."""
        off = torch.empty(self.n_grid + 1, dtype=torch.int32, device=self.device)
        adj = torch.empty(max(1, 8 * self.n_voxels), dtype=torch.int32, device=self.device)
        nb = _abi.svr_grid_adjacency_scratch_bytes(self.n_voxels, self.n_grid)
        scratch = torch.empty(nb + 256, dtype=torch.uint8, device=self.device)
        p = (scratch.data_ptr() + 255) // 256 * 256
        check(_abi.svr_build_grid_adjacency(_ptr(self.vox_grid), self.n_voxels, self.n_grid,
                                            _ptr(off), _ptr(adj), ctypes.c_void_p(p), nb,
                                            _stream()), "svr_build_grid_adjacency")
        torch.cuda.current_stream().synchronize()
        del scratch
        self.adj_off, self.adj = off, adj

    def nbytes(self) -> int:
        """Device bytes of the scene arrays (adjacency included)."""
        ts = [self.center, self.size, self.octpath, self.vox_grid, self.grid_raw, self.sh,
              self.adj_off, self.adj, self.rank]
        return int(sum(t.numel() * t.element_size() for t in ts if t is not None))

    def struct(self, grid_raw: Optional[torch.Tensor] = None,
               sh: Optional[torch.Tensor] = None) -> _abi.svr_scene:
        g = self.grid_raw if grid_raw is None else grid_raw
        s = self.sh if sh is None else sh
        for t, name in ((g, "grid_raw"), (s, "sh")):
            if t.dtype != torch.float32 or not t.is_contiguous() or t.device != self.device:
                raise ValueError("%s must be a contiguous float32 tensor on %s" % (name, self.device))
        if g.numel() != self.n_grid or s.numel() != self.n_voxels * 3 * (self.sh_degree + 1) ** 2:
            raise ValueError("grid_raw / sh sizes do not match the scene")
        st = _abi.svr_scene()
        st.n_voxels = self.n_voxels
        st.n_grid = self.n_grid
        st.center = self.center.data_ptr()
        st.size = self.size.data_ptr()
        st.octpath = self.octpath.data_ptr()
        st.vox_grid = self.vox_grid.data_ptr()
        st.grid_raw = g.data_ptr()
        st.sh = s.data_ptr()
        st.sh_degree = self.sh_degree
        st.max_level = self.max_level
        if self.adj_off is not None:
            st.grid_adj_off = self.adj_off.data_ptr()
            st.grid_adj = self.adj.data_ptr()
        if self.rank is not None:
            st.order_rank = self.rank.data_ptr()
        return st


def camera_structs(cams: Sequence) -> ctypes.Array:
    arr = (_abi.svr_camera * len(cams))()
    for i, c in enumerate(cams):
        arr[i].width = int(c.W)
        arr[i].height = int(c.H)
        arr[i].fx = float(c.fx)
        arr[i].fy = float(c.fy)
        arr[i].cx = float(c.cx)
        arr[i].cy = float(c.cy)
        w = np.asarray(c.w2c, np.float32).reshape(-1)
        for k in range(12):
            arr[i].w2c[k] = float(w[k])
    return arr


class Rasterizer:
    """One frame of one or more cameras over a device scene.

    ``forward()`` runs svr_preprocess, svr_sort and svr_render_fwd and returns
    rgba of shape (sum H*W, 4); ``backward(grad_rgba)`` runs svr_render_bwd on
    the same workspace.  ``sync_count`` reads the entry count back once per
    frame (exact capacity check, sort sized to the count); without it the
    frame has no host synchronisation and overflow is checked afterwards.
    """

    def __init__(self, dscene: DeviceScene, cams: Sequence, K: int = 1, t_stop: float = 1e-4,
                 activation: int = _abi.SVR_ACT_EXPLIN, capacity: Optional[int] = None,
                 sync_count: bool = True, tile: int = 16, persistent: int = 0,
                 accumulate: bool = False):
        if len(cams) < 1 or len(cams) > _abi.SVR_MAX_CAMERAS:
            raise ValueError("1..%d cameras per frame" % _abi.SVR_MAX_CAMERAS)
        self.ds = dscene
        self.cams = list(cams)
        self.cam_arr = camera_structs(self.cams)
        self.n_cams = len(self.cams)
        self.n_pixels = int(sum(c.W * c.H for c in self.cams))
        self.opts = _abi.svr_opts()
        self.opts.K = int(K)
        self.opts.t_stop = float(t_stop)
        self.opts.activation = int(activation)
        self.opts.tile = int(tile)
        self.opts.persistent = int(persistent)
        self.opts.accumulate = 1 if accumulate else 0
        self._graph = None
        self._view_graphs = []
        if capacity is None:
            capacity = max(1 << 16, 2 * dscene.n_voxels * self.n_cams)
        self.sync_count = sync_count
        self.n_entries = -1
        # bumped by every preprocess: the workspace holds the lists of the
        # frame with this number
        self.frame = 0
        self.ws = None
        self.ws_bytes = 0
        self._set_capacity(int(capacity))

    def _set_capacity(self, cap: int):
        cap = min(cap, (1 << 30) - 1)
        self.opts.entry_capacity = cap
        st = self.ds.struct()
        nb = _abi.svr_workspace_bytes(st, self.cam_arr, self.n_cams, self.opts)
        if nb == 0:
            raise ValueError("invalid rasterizer configuration: " + _abi.svr_last_error())
        if self.ws is None or self.ws_bytes < nb:
            self.ws = None
            self.ws = torch.empty(nb + 256, dtype=torch.uint8, device=self.ds.device)
            self.ws_bytes = nb
        self.capacity = cap

    def workspace_parts(self) -> dict:
        """Bytes of this frame's workspace by purpose (svr_workspace_parts)."""
        return _abi.svr_workspace_parts(self.ds.struct(), self.cam_arr, self.n_cams, self.opts)

    def _ws_ptr(self):
        p = self.ws.data_ptr()
        p = (p + 255) // 256 * 256
        return ctypes.c_void_p(p)

    def workspace_bytes(self) -> int:
        return self.ws_bytes

    def preprocess(self, grid_raw=None, sh=None):
        st = self.ds.struct(grid_raw, sh)
        self.frame += 1
        if self.sync_count:
            n = ctypes.c_int64(0)
            rc = _abi.svr_preprocess(st, self.cam_arr, self.n_cams, self.opts, self._ws_ptr(),
                                     self.ws_bytes, ctypes.byref(n), _stream())
            if rc == _abi.SVR_E_CAPACITY:
                self._set_capacity(int(n.value * 1.25) + 1024)
                rc = _abi.svr_preprocess(st, self.cam_arr, self.n_cams, self.opts, self._ws_ptr(),
                                         self.ws_bytes, ctypes.byref(n), _stream())
            check(rc, "svr_preprocess")
            self.n_entries = int(n.value)
        else:
            check(_abi.svr_preprocess(st, self.cam_arr, self.n_cams, self.opts, self._ws_ptr(),
                                      self.ws_bytes, None, _stream()), "svr_preprocess")
            self.n_entries = -1

    def sort(self):
        st = self.ds.struct()
        check(_abi.svr_sort(st, self.cam_arr, self.n_cams, self.opts, self._ws_ptr(),
                            self.ws_bytes, self.n_entries, _stream()), "svr_sort")

    def render_fwd(self, grid_raw=None, sh=None, out: Optional[torch.Tensor] = None,
                   max_weight: Optional[torch.Tensor] = None,
                   depth: Optional[torch.Tensor] = None, normal: Optional[torch.Tensor] = None):
        """``max_weight`` (float32 [n_voxels], zeroed by the caller once per
        statistics window): per-voxel maximum blending weight, updated.
        ``depth`` [n_pixels] / ``normal`` [n_pixels, 3]: depth and normal
        images, written."""
        st = self.ds.struct(grid_raw, sh)
        if out is None:
            out = torch.empty((self.n_pixels, 4), dtype=torch.float32, device=self.ds.device)
        ex = _extra(max_weight=max_weight, depth=depth, normal=normal)
        check(_abi.svr_render_fwd(st, self.cam_arr, self.n_cams, self.opts, self._ws_ptr(),
                                  self.ws_bytes, _ptr(out), ex, _stream()), "svr_render_fwd")
        return out

    def forward(self, grid_raw=None, sh=None, out=None, max_weight=None, depth=None,
                normal=None):
        self.preprocess(grid_raw, sh)
        self.sort()
        return self.render_fwd(grid_raw, sh, out, max_weight, depth, normal)

    def backward(self, grad_rgba: torch.Tensor, grid_raw=None, sh=None, grad_grid=None,
                 grad_sh=None, want_grid=True, want_sh=True,
                 priority: Optional[torch.Tensor] = None,
                 grad_depth: Optional[torch.Tensor] = None,
                 grad_normal: Optional[torch.Tensor] = None):
        """``priority`` (float32 [n_voxels]): per-voxel subdivision priority,
        accumulated into.  ``grad_depth`` / ``grad_normal``: upstream gradients
        of the depth and normal images (the forward must have produced them)."""
        st = self.ds.struct(grid_raw, sh)
        g = grad_rgba.contiguous().float()
        if g.numel() != self.n_pixels * 4:
            raise ValueError("grad_rgba must have shape (n_pixels, 4)")
        if want_grid and grad_grid is None:
            grad_grid = torch.empty(self.ds.n_grid, dtype=torch.float32, device=self.ds.device)
        if want_sh and grad_sh is None:
            grad_sh = torch.empty_like(self.ds.sh)
        check(_abi.svr_render_bwd(st, self.cam_arr, self.n_cams, self.opts, self._ws_ptr(),
                                  self.ws_bytes, _ptr(g), _ptr(grad_grid if want_grid else None),
                                  _ptr(grad_sh if want_sh else None),
                                  _extra(priority=priority, grad_depth=grad_depth,
                                         grad_normal=grad_normal),
                                  _stream()),
              "svr_render_bwd")
        return grad_grid, grad_sh

    # -- whole-frame hipGraph ----------------------------------------------------
    def capture(self, rgba: torch.Tensor, grad_rgba: Optional[torch.Tensor] = None,
                grad_grid: Optional[torch.Tensor] = None, grad_sh: Optional[torch.Tensor] = None,
                stream: Optional[torch.cuda.Stream] = None):
        """Capture preprocess + sort + fwd (+ bwd) of this frame into a hipGraph
        that writes the given tensors at every replay."""
        self.release_graph()
        stream = stream or torch.cuda.Stream()
        st = self.ds.struct()
        h = ctypes.c_void_p(0)
        torch.cuda.synchronize()
        check(_abi.svr_graph_capture(st, self.cam_arr, self.n_cams, self.opts, self._ws_ptr(),
                                     self.ws_bytes, _ptr(rgba), _ptr(grad_rgba), _ptr(grad_grid),
                                     _ptr(grad_sh), None, ctypes.c_void_p(stream.cuda_stream),
                                     ctypes.byref(h)), "svr_graph_capture")
        self._graph = h
        self._graph_keep = (rgba, grad_rgba, grad_grid, grad_sh)
        return h

    def replay(self, stream: Optional[torch.cuda.Stream] = None):
        s = (stream or torch.cuda.current_stream()).cuda_stream
        self.frame += 1
        check(_abi.svr_graph_launch(self._graph, ctypes.c_void_p(s)), "svr_graph_launch")

    def capture_views(self, cams: Sequence, rgba: torch.Tensor, grad_rgba: torch.Tensor,
                      grad_grid: torch.Tensor, grad_sh: torch.Tensor,
                      stream: torch.cuda.Stream) -> int:
        """One hipGraph per camera (each of this rasterizer's resolution), all
        sharing this workspace and the given outputs: replay_view(i) runs the
        whole frame of camera i.  Replays must run one after another on one
        stream.  Returns the number of graphs."""
        self.release_graph()
        st = self.ds.struct()
        for c in cams:
            self.set_cameras([c])
            h = ctypes.c_void_p(0)
            torch.cuda.synchronize()
            check(_abi.svr_graph_capture(st, self.cam_arr, self.n_cams, self.opts,
                                         self._ws_ptr(), self.ws_bytes, _ptr(rgba),
                                         _ptr(grad_rgba), _ptr(grad_grid), _ptr(grad_sh), None,
                                         ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h)),
                  "svr_graph_capture")
            self._view_graphs.append(h)
        self._graph_keep = (rgba, grad_rgba, grad_grid, grad_sh)
        return len(self._view_graphs)

    def replay_view(self, i: int, stream: torch.cuda.Stream):
        self.frame += 1
        check(_abi.svr_graph_launch(self._view_graphs[i], ctypes.c_void_p(stream.cuda_stream)),
              "svr_graph_launch")

    def release_graph(self):
        if self._graph is not None:
            _abi.svr_graph_destroy(self._graph)
            self._graph = None
        for h in self._view_graphs:
            _abi.svr_graph_destroy(h)
        self._view_graphs = []

    def __del__(self):
        try:
            self.release_graph()
        except Exception:
            pass

    def set_cameras(self, cams: Sequence):
        """Swap in cameras of the same resolutions (workspace size unchanged)."""
        if len(cams) != self.n_cams or any((a.W, a.H) != (b.W, b.H) for a, b in zip(cams, self.cams)):
            raise ValueError("set_cameras needs the same number and sizes of cameras")
        self.cams = list(cams)
        self.cam_arr = camera_structs(self.cams)

    def stats(self):
        """(entries, walked pixel-entry pairs, executed ray-box tests, hits,
        in-view voxels)."""
        st = self.ds.struct()
        counts = (ctypes.c_int64 * 5)()
        check(_abi.svr_render_stats(st, self.cam_arr, self.n_cams, self.opts, self._ws_ptr(),
                                    self.ws_bytes, counts, _stream()), "svr_render_stats")
        return tuple(int(x) for x in counts)

    def check_overflow(self) -> int:
        st = self.ds.struct()
        n = ctypes.c_int64(0)
        rc = _abi.svr_check_overflow(st, self.cam_arr, self.n_cams, self.opts, self._ws_ptr(),
                                     self.ws_bytes, ctypes.byref(n), _stream())
        if rc == _abi.SVR_E_CAPACITY:
            return int(n.value)
        check(rc, "svr_check_overflow")
        return int(n.value)

    def sorted_entries(self, n: int):
        keys = torch.empty(max(n, 1), dtype=torch.int64, device=self.ds.device)
        vals = torch.empty(max(n, 1), dtype=torch.int32, device=self.ds.device)
        st = self.ds.struct()
        check(_abi.svr_copy_sorted(st, self.cam_arr, self.n_cams, self.opts, self._ws_ptr(),
                                   self.ws_bytes, _ptr(keys), _ptr(vals), n, _stream()),
              "svr_copy_sorted")
        return keys[:n], vals[:n]


class BatchRenderer:
    """Forward + backward of many cameras (any mix of resolutions) as groups of
    `group` cameras, each group one hipGraph (one launch per stage for all its
    cameras); the gradients of all groups accumulate into one pair of buffers.
    """

    def __init__(self, dscene: DeviceScene, cams: Sequence, K: int, group: int, tile: int = 16,
                 persistent: int = 0, activation: int = _abi.SVR_ACT_EXPLIN,
                 t_stop: float = 1e-4, slack: float = 1.1):
        self.ds = dscene
        self.cams = list(cams)
        self.group = max(1, min(int(group), len(self.cams), _abi.SVR_MAX_CAMERAS))
        self.groups = [self.cams[i:i + self.group] for i in range(0, len(self.cams), self.group)]
        self.n_pixels = int(sum(c.W * c.H for c in self.cams))
        dev = dscene.device
        self.rgba = torch.empty((self.n_pixels, 4), dtype=torch.float32, device=dev)
        self.grad_grid = torch.empty(dscene.n_grid, dtype=torch.float32, device=dev)
        self.grad_sh = torch.empty_like(dscene.sh)
        self.rasts = []
        off = 0
        for gi, gc in enumerate(self.groups):
            probe = Rasterizer(dscene, gc, K=K, t_stop=t_stop, activation=activation,
                               sync_count=True, tile=tile)
            probe.preprocess()
            cap = int(probe.n_entries * slack) + 4096
            del probe
            r = Rasterizer(dscene, gc, K=K, t_stop=t_stop, activation=activation, capacity=cap,
                           sync_count=False, tile=tile, persistent=persistent,
                           accumulate=gi > 0)
            npx = r.n_pixels
            r._rows = (off, off + npx)
            off += npx
            self.rasts.append(r)
        self.stream = torch.cuda.Stream()

    def workspace_bytes(self) -> int:
        return int(sum(r.ws_bytes for r in self.rasts))

    def workspace_parts(self) -> dict:
        tot: dict = {}
        for r in self.rasts:
            for k, v in r.workspace_parts().items():
                tot[k] = tot.get(k, 0) + v
        return tot

    def capture(self, grad_rgba: torch.Tensor):
        self.grad_rgba = grad_rgba.contiguous()
        for r in self.rasts:
            a, b = r._rows
            r.capture(self.rgba[a:b], self.grad_rgba[a:b], self.grad_grid, self.grad_sh,
                      self.stream)

    def replay(self):
        for r in self.rasts:
            r.replay(self.stream)

    def check_overflow(self) -> bool:
        ok = True
        for r in self.rasts:
            ok &= r.check_overflow() <= r.capacity
        return ok


class SVRasterFunction(torch.autograd.Function):
    """rgba = render(grid_raw, sh) for a fixed rasterizer (scene geometry and
    cameras); gradients flow to the corner raw densities and SH coefficients.

    The adjoint reads the sorted lists and per-pixel state the forward left
    in the rasterizer's workspace.  When another frame has gone through the
    same rasterizer since this forward (a second render before backward,
    activation checkpointing), the backward first renders this frame again
    from the saved parameters and cameras, so the gradients always belong
    to the forward they differentiate."""

    @staticmethod
    def forward(ctx, grid_raw, sh, rast: Rasterizer):
        grid_raw = grid_raw.contiguous()
        sh = sh.contiguous()
        rgba = rast.forward(grid_raw, sh)
        ctx.rast = rast
        ctx.frame = rast.frame
        ctx.cams = list(rast.cams)
        ctx.save_for_backward(grid_raw, sh)
        return rgba

    @staticmethod
    def backward(ctx, grad_rgba):
        grid_raw, sh = ctx.saved_tensors
        rast = ctx.rast
        cams_now = None
        if rast.frame != ctx.frame:
            cams_now = list(rast.cams)
            rast.set_cameras(ctx.cams)
            rast.forward(grid_raw, sh)
        gg, gs = rast.backward(grad_rgba, grid_raw, sh,
                               want_grid=ctx.needs_input_grad[0],
                               want_sh=ctx.needs_input_grad[1])
        if cams_now is not None:
            rast.set_cameras(cams_now)
        return gg, gs, None


def render(rast: Rasterizer, grid_raw: torch.Tensor, sh: torch.Tensor) -> torch.Tensor:
    return SVRasterFunction.apply(grid_raw, sh, rast)


def radix_sort_pairs(keys: torch.Tensor, vals: torch.Tensor, bits: int = 64):
    """Sort int64 (read as uint64) keys with int32 values in place on the GPU."""
    n = keys.numel()
    if n == 0:
        return keys, vals
    kt = torch.empty_like(keys)
    vt = torch.empty_like(vals)
    nb = _abi.svr_radix_sort_scratch_bytes(n, bits)
    scratch = torch.empty(nb + 256, dtype=torch.uint8, device=keys.device)
    p = (scratch.data_ptr() + 255) // 256 * 256
    check(_abi.svr_radix_sort_pairs(_ptr(keys), _ptr(vals), _ptr(kt), _ptr(vt), n, bits,
                                    ctypes.c_void_p(p), nb, _stream()), "svr_radix_sort_pairs")
    return keys, vals


# -- anti-aliasing (Sec. 3.1.2 "Anti-aliasing") and background -----------------------
def supersampled_camera(cam, ss: float):
    """The camera rendering ``cam``'s view at ss times its resolution
    (rounded), intrinsics scaled with the image so that pixel centres map
    onto each other: (u + 1/2) W' / W."""
    import dataclasses
    W2 = max(cam.W, int(round(cam.W * ss)))
    H2 = max(cam.H, int(round(cam.H * ss)))
    sx, sy = W2 / cam.W, H2 / cam.H
    return dataclasses.replace(cam, W=W2, H=H2, fx=cam.fx * sx, fy=cam.fy * sy, cx=cam.cx * sx,
                               cy=cam.cy * sy)


def _bg_arr(bg):
    if bg is None:
        return None
    a = (ctypes.c_float * 3)(*[float(x) for x in bg])
    return a


class DownsampleFunction(torch.autograd.Function):
    """rgba at (w_out, h_out) from a supersampled rgba (svr_downsample), with
    the background colour bg composited behind; differentiable in the input."""

    @staticmethod
    def forward(ctx, rgba_in, w_in, h_in, w_out, h_out, bg):
        x = rgba_in.contiguous()
        out = torch.empty((w_out * h_out, 4), dtype=torch.float32, device=x.device)
        check(_abi.svr_downsample(_ptr(x), w_in, h_in, _ptr(out), w_out, h_out, _bg_arr(bg),
                                  _stream()), "svr_downsample")
        ctx.sizes = (w_in, h_in, w_out, h_out)
        ctx.bg = bg
        return out

    @staticmethod
    def backward(ctx, grad_out):
        w_in, h_in, w_out, h_out = ctx.sizes
        g = grad_out.contiguous().float()
        gin = torch.empty((w_in * h_in, 4), dtype=torch.float32, device=g.device)
        check(_abi.svr_downsample_bwd(_ptr(g), w_out, h_out, _ptr(gin), w_in, h_in,
                                      _bg_arr(ctx.bg), _stream()), "svr_downsample_bwd")
        return gin, None, None, None, None, None


def downsample(rgba_in: torch.Tensor, w_in: int, h_in: int, w_out: int, h_out: int, bg=None):
    """Anti-aliased downsample of a supersampled render plus background."""
    return DownsampleFunction.apply(rgba_in, w_in, h_in, w_out, h_out, bg)


# ---------------------------------------------------------------------------
# Mesh extraction (Sec. 3.2.4): TSDF fusion of rendered depths at the grid
# points, then marching cubes over the voxels.

def _f32_dev(t, name, n=None):
    if t.dtype != torch.float32 or not t.is_contiguous() or t.device.type != "cuda":
        raise ValueError("%s must be a contiguous float32 device tensor" % name)
    if n is not None and t.numel() != n:
        raise ValueError("%s has %d elements, expected %d" % (name, t.numel(), n))
    return t


def morton_order(pos: torch.Tensor, lo, extent: float) -> torch.Tensor:
    """Z-curve visit order (int32 [n]) of the points pos (float32 [3, n]) in
    the cube [lo, lo + extent): svr_morton_keys, then svr_radix_sort_pairs on
    the 30 key bits."""
    if pos.dim() != 2 or pos.shape[0] != 3:
        raise ValueError("pos must be [3, n]")
    n = pos.shape[1]
    _f32_dev(pos, "pos", 3 * n)
    keys = torch.empty(max(n, 1), dtype=torch.int64, device=pos.device)
    vals = torch.empty(max(n, 1), dtype=torch.int32, device=pos.device)
    lo3 = (ctypes.c_float * 3)(*[float(x) for x in lo])
    check(_abi.svr_morton_keys(_ptr(pos), n, lo3, float(extent), _ptr(keys), _ptr(vals),
                               _stream()), "svr_morton_keys")
    radix_sort_pairs(keys[:n], vals[:n], bits=30)
    return vals[:n]


def tsdf_fuse(grid_pos: torch.Tensor, cams: Sequence, depth: torch.Tensor, trunc: float,
              rgba: Optional[torch.Tensor] = None, min_alpha: float = 0.5,
              tsdf: Optional[torch.Tensor] = None, weight: Optional[torch.Tensor] = None,
              order: Optional[torch.Tensor] = None):
    """Fused truncated signed distances (svr_tsdf_fuse).  grid_pos float32
    [3, M]; depth [sum H*W] of the cameras in order (with ``rgba``: the
    renderer's composited depth, divided by the opacity where it reaches
    ``min_alpha``); ``order`` (int32 [M]): visit order of the grid points
    (``morton_order``), None for their own order.  Returns (tsdf [M],
    weight [M])."""
    if grid_pos.dim() != 2 or grid_pos.shape[0] != 3:
        raise ValueError("grid_pos must be [3, M] (x row, y row, z row)")
    M = grid_pos.shape[1]
    _f32_dev(grid_pos, "grid_pos", 3 * M)
    P = int(sum(c.W * c.H for c in cams))
    _f32_dev(depth, "depth", P)
    if rgba is not None:
        _f32_dev(rgba, "rgba", 4 * P)
    if tsdf is None:
        tsdf = torch.empty(M, dtype=torch.float32, device=grid_pos.device)
    if weight is None:
        weight = torch.empty(M, dtype=torch.float32, device=grid_pos.device)
    _f32_dev(tsdf, "tsdf", M)
    _f32_dev(weight, "weight", M)
    _check_order(order, M, grid_pos.device)
    arr = camera_structs(cams)
    check(_abi.svr_tsdf_fuse(_ptr(grid_pos), M, arr, len(cams), _ptr(depth), _ptr(rgba),
                             float(min_alpha), float(trunc), _ptr(tsdf), _ptr(weight),
                             _ptr(order), _stream()), "svr_tsdf_fuse")
    return tsdf, weight


def _check_order(order, n, device):
    if order is None:
        return
    if (order.dtype != torch.int32 or order.numel() != n or not order.is_contiguous()
            or order.device != device):
        raise ValueError("order must be a contiguous int32 tensor of %d entries on %s"
                         % (n, device))


def marching_cubes_into(ds: DeviceScene, field: torch.Tensor, keys: torch.Tensor,
                        pos: torch.Tensor, count: torch.Tensor, iso: float = 0.0,
                        weight: Optional[torch.Tensor] = None,
                        order: Optional[torch.Tensor] = None):
    """svr_marching_cubes into preallocated keys int32 [cap, 3, 2], pos float32
    [cap, 3, 3] and count int64 [1] (the total, which may exceed cap); no
    host synchronisation."""
    _f32_dev(field, "field", ds.n_grid)
    if weight is not None:
        _f32_dev(weight, "weight", ds.n_grid)
    cap = keys.shape[0]
    if keys.dtype != torch.int32 or tuple(keys.shape[1:]) != (3, 2) or not keys.is_contiguous():
        raise ValueError("keys must be a contiguous int32 [cap, 3, 2] tensor")
    if pos.dtype != torch.float32 or tuple(pos.shape) != (cap, 3, 3) or not pos.is_contiguous():
        raise ValueError("pos must be a contiguous float32 [cap, 3, 3] tensor")
    if count.dtype != torch.int64 or count.numel() != 1:
        raise ValueError("count must be an int64 tensor of one element")
    _check_order(order, ds.n_voxels, ds.device)
    st = ds.struct()
    check(_abi.svr_marching_cubes(st, _ptr(field), _ptr(weight), float(iso), cap, _ptr(keys),
                                  _ptr(pos), _ptr(count), _ptr(order), _stream()),
          "svr_marching_cubes")


def marching_cubes(ds: DeviceScene, field: torch.Tensor, iso: float = 0.0,
                   weight: Optional[torch.Tensor] = None, capacity: Optional[int] = None,
                   order: Optional[torch.Tensor] = None):
    """Iso-surface triangles over the voxels (svr_marching_cubes): (keys int32
    [n, 3, 2] grid point pairs per vertex, pos float32 [n, 3, 3]).  The
    triangle order is not deterministic."""
    dev = ds.device
    cap = max(1024, ds.n_voxels // 2) if capacity is None else int(capacity)
    count = torch.zeros(1, dtype=torch.int64, device=dev)
    for _ in range(2):
        keys = torch.empty((cap, 3, 2), dtype=torch.int32, device=dev)
        pos = torch.empty((cap, 3, 3), dtype=torch.float32, device=dev)
        marching_cubes_into(ds, field, keys, pos, count, iso, weight, order)
        n = int(count.item())
        if n <= cap:
            return keys[:n], pos[:n]
        cap = n
    raise RuntimeError("marching cubes: triangle count changed between calls")


def mesh_case_table():
    """The cell table of svr_marching_cubes: (counts uint8 [256], verts uint8
    [256, 36]) with vertices as corner pairs a << 3 | b."""
    counts = (ctypes.c_uint8 * 256)()
    verts = (ctypes.c_uint8 * (256 * 36))()
    check(_abi.svr_mesh_case_table(counts, verts), "svr_mesh_case_table")
    return (np.frombuffer(counts, np.uint8).copy(),
            np.frombuffer(verts, np.uint8).reshape(256, 36).copy())
