"""ctypes binding of ``include/svraster.h`` (argument marshalling only).

The functions below carry the C names and pass their arguments straight
through; every step of the rendering runs in ``lib/libsvraster.so``.  The
library is loaded on first use and a missing library is an error, never a
fallback.  When torch is importable it is imported first so that the
library binds to the HIP runtime torch already uses.
"""
from __future__ import annotations

import ctypes
import os
import re

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "lib", "libsvraster.so")
HEADER_PATH = os.path.join(os.path.dirname(_PKG), "include", "svraster.h")

SVR_OK = 0
SVR_E_INVALID = -1
SVR_E_CAPACITY = -2
SVR_E_HIP = -3
SVR_E_WORKSPACE = -4
SVR_E_DEVICE = -5
SVR_ACT_EXPLIN = 0
SVR_ACT_SOFTPLUS = 1
SVR_MAX_CAMERAS = 32
SVR_TILE = 16
SVR_STATIC_SORT_MAX = 1 << 21

P = ctypes.c_void_p
I64 = ctypes.c_int64
I32 = ctypes.c_int32


class svr_scene(ctypes.Structure):
    _fields_ = [("n_voxels", I64), ("n_grid", I64), ("center", P), ("size", P), ("octpath", P),
                ("vox_grid", P), ("grid_raw", P), ("sh", P), ("sh_degree", I32),
                ("max_level", I32), ("grid_adj_off", P), ("grid_adj", P), ("order_rank", P)]


class svr_camera(ctypes.Structure):
    _fields_ = [("width", I32), ("height", I32), ("fx", ctypes.c_float), ("fy", ctypes.c_float),
                ("cx", ctypes.c_float), ("cy", ctypes.c_float), ("w2c", ctypes.c_float * 12)]


class svr_opts(ctypes.Structure):
    _fields_ = [("K", I32), ("t_stop", ctypes.c_float), ("activation", I32), ("tile", I32),
                ("entry_capacity", I64), ("persistent", I32), ("accumulate", I32)]


class svr_extra(ctypes.Structure):
    _fields_ = [("max_weight", ctypes.c_void_p), ("priority", ctypes.c_void_p),
                ("depth", ctypes.c_void_p), ("normal", ctypes.c_void_p),
                ("grad_depth", ctypes.c_void_p), ("grad_normal", ctypes.c_void_p)]


_SIGS = {
    "svr_workspace_bytes": (ctypes.c_size_t, [P, P, ctypes.c_int, P]),
    "svr_workspace_parts": (ctypes.c_int, [P, P, ctypes.c_int, P, P, ctypes.c_int]),
    "svr_preprocess": (ctypes.c_int, [P, P, ctypes.c_int, P, P, ctypes.c_size_t, P, P]),
    "svr_sort": (ctypes.c_int, [P, P, ctypes.c_int, P, P, ctypes.c_size_t, I64, P]),
    "svr_render_fwd": (ctypes.c_int, [P, P, ctypes.c_int, P, P, ctypes.c_size_t, P, P, P]),
    "svr_render_bwd": (ctypes.c_int, [P, P, ctypes.c_int, P, P, ctypes.c_size_t, P, P, P, P, P]),
    "svr_check_overflow": (ctypes.c_int, [P, P, ctypes.c_int, P, P, ctypes.c_size_t, P, P]),
    "svr_copy_sorted": (ctypes.c_int, [P, P, ctypes.c_int, P, P, ctypes.c_size_t, P, P, I64, P]),
    "svr_radix_sort_scratch_bytes": (ctypes.c_size_t, [I64, ctypes.c_int]),
    "svr_radix_sort_pairs": (ctypes.c_int, [P, P, P, P, I64, ctypes.c_int, P, ctypes.c_size_t, P]),
    "svr_radix_sort_pairs_static": (ctypes.c_int, [P, P, I64, ctypes.c_int, P]),
    "svr_atomic_probe": (ctypes.c_int, [P, P, I64, I64, ctypes.c_int, P]),
    "svr_render_stats": (ctypes.c_int, [P, P, ctypes.c_int, P, P, ctypes.c_size_t, P, P]),
    "svr_timing_enable": (ctypes.c_int, [ctypes.c_int]),
    "svr_timing_read": (ctypes.c_int, [P, ctypes.c_int, P, P, ctypes.c_int, P]),
    "svr_graph_capture": (ctypes.c_int, [P, P, ctypes.c_int, P, P, ctypes.c_size_t, P, P, P, P, P,
                                         P, P]),
    "svr_graph_launch": (ctypes.c_int, [P, P]),
    "svr_order_rank_scratch_bytes": (ctypes.c_size_t, [I64, ctypes.c_int]),
    "svr_build_order_ranks": (ctypes.c_int, [P, I64, ctypes.c_int, P, P, ctypes.c_size_t, P]),
    "svr_downsample": (ctypes.c_int, [P, ctypes.c_int, ctypes.c_int, P, ctypes.c_int, ctypes.c_int,
                                      P, P]),
    "svr_downsample_bwd": (ctypes.c_int, [P, ctypes.c_int, ctypes.c_int, P, ctypes.c_int,
                                          ctypes.c_int, P, P]),
    "svr_graph_destroy": (ctypes.c_int, [P]),
    "svr_tsdf_fuse": (ctypes.c_int, [P, I64, P, ctypes.c_int, P, P, ctypes.c_float, ctypes.c_float,
                                     P, P, P, P]),
    "svr_marching_cubes": (ctypes.c_int, [P, P, P, ctypes.c_float, I64, P, P, P, P, P]),
    "svr_morton_keys": (ctypes.c_int, [P, I64, P, ctypes.c_float, P, P, P]),
    "svr_mesh_case_table": (ctypes.c_int, [P, P]),
    "svr_grid_adjacency_scratch_bytes": (ctypes.c_size_t, [I64, I64]),
    "svr_build_grid_adjacency": (ctypes.c_int, [P, I64, I64, P, P, P, ctypes.c_size_t, P]),
    "svr_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "svr_last_error": (ctypes.c_char_p, []),
}

_lib = None


def header_functions():
    """Names of the functions declared in include/svraster.h."""
    text = open(HEADER_PATH).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(svr_[a-z_0-9]+)\s*\(", text)))


def load(with_torch: bool = True):
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                "libsvraster.so is not built (%s); run `python -m paper_2412_04459_amd.build`"
                % LIB_PATH)
        if with_torch:
            try:
                import torch  # noqa: F401  share torch's HIP runtime
            except ImportError:
                pass
        lib = ctypes.CDLL(LIB_PATH, mode=ctypes.RTLD_GLOBAL)
        for name, (res, args) in _SIGS.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def _ref(x):
    return None if x is None else ctypes.byref(x)


class SvrError(RuntimeError):
    def __init__(self, status, where):
        lib = load()
        msg = "%s failed: %s (%s)" % (where, lib.svr_status_string(status).decode(),
                                     lib.svr_last_error().decode())
        super().__init__(msg)
        self.status = status


def check(status, where):
    if status == SVR_OK:
        return
    if status == SVR_E_INVALID:
        lib = load()
        raise ValueError("%s: %s" % (where, lib.svr_last_error().decode()))
    raise SvrError(status, where)


# -- thin pass-throughs with the C names --------------------------------------
def svr_workspace_bytes(scene, cams, n_cams, opts):
    return load().svr_workspace_bytes(_ref(scene), cams, n_cams, _ref(opts))


SVR_WS_PARTS = 7
WS_PART_NAMES = ("header_and_tile_tables", "per_voxel_camera_records", "scan_partials",
                 "keys_values_x2", "sort_histograms_and_status", "per_pixel_state",
                 "gradient_scratch")


def svr_workspace_parts(scene, cams, n_cams, opts):
    """Workspace bytes by purpose, as a dict keyed by WS_PART_NAMES."""
    arr = (ctypes.c_size_t * SVR_WS_PARTS)()
    check(load().svr_workspace_parts(_ref(scene), cams, n_cams, _ref(opts), arr, SVR_WS_PARTS),
          "svr_workspace_parts")
    return dict(zip(WS_PART_NAMES, (int(x) for x in arr)))


def svr_preprocess(scene, cams, n_cams, opts, ws, ws_bytes, n_entries_out, stream):
    return load().svr_preprocess(_ref(scene), cams, n_cams, _ref(opts), ws, ws_bytes,
                                 n_entries_out, stream)


def svr_sort(scene, cams, n_cams, opts, ws, ws_bytes, n_entries_hint, stream):
    return load().svr_sort(_ref(scene), cams, n_cams, _ref(opts), ws, ws_bytes, n_entries_hint,
                           stream)


def svr_render_fwd(scene, cams, n_cams, opts, ws, ws_bytes, rgba, extra, stream):
    return load().svr_render_fwd(_ref(scene), cams, n_cams, _ref(opts), ws, ws_bytes, rgba,
                                 _ref(extra), stream)


def svr_render_bwd(scene, cams, n_cams, opts, ws, ws_bytes, grad_rgba, grad_grid, grad_sh, extra,
                   stream):
    return load().svr_render_bwd(_ref(scene), cams, n_cams, _ref(opts), ws, ws_bytes, grad_rgba,
                                 grad_grid, grad_sh, _ref(extra), stream)


def svr_check_overflow(scene, cams, n_cams, opts, ws, ws_bytes, required_entries, stream):
    return load().svr_check_overflow(_ref(scene), cams, n_cams, _ref(opts), ws, ws_bytes,
                                     required_entries, stream)


def svr_copy_sorted(scene, cams, n_cams, opts, ws, ws_bytes, keys, values, n, stream):
    return load().svr_copy_sorted(_ref(scene), cams, n_cams, _ref(opts), ws, ws_bytes, keys,
                                  values, n, stream)


def svr_radix_sort_scratch_bytes(n, bits):
    return load().svr_radix_sort_scratch_bytes(n, bits)


def svr_radix_sort_pairs(keys, values, keys_tmp, values_tmp, n, bits, scratch, scratch_bytes,
                         stream):
    return load().svr_radix_sort_pairs(keys, values, keys_tmp, values_tmp, n, bits, scratch,
                                       scratch_bytes, stream)


def svr_radix_sort_pairs_static(keys, values, n, bits, stream):
    return load().svr_radix_sort_pairs_static(keys, values, n, bits, stream)


def svr_atomic_probe(corner, colour, n_rows, n_waves, iters, stream):
    return load().svr_atomic_probe(corner, colour, n_rows, n_waves, iters, stream)


def svr_render_stats(scene, cams, n_cams, opts, ws, ws_bytes, counts, stream):
    return load().svr_render_stats(_ref(scene), cams, n_cams, _ref(opts), ws, ws_bytes, counts,
                                   stream)


def svr_timing_enable(on):
    return load().svr_timing_enable(int(on))


def svr_timing_read(names, name_len, total_ms, launches, max_n, n_out):
    return load().svr_timing_read(names, name_len, total_ms, launches, max_n, n_out)


def kernel_times():
    """{kernel name: (total ms, launches)} since the last read (timing must be on)."""
    n_max, L = 64, 48
    names = ctypes.create_string_buffer(n_max * L)
    ms = (ctypes.c_double * n_max)()
    cnt = (ctypes.c_int64 * n_max)()
    n = ctypes.c_int(0)
    check(load().svr_timing_read(names, L, ms, cnt, n_max, ctypes.byref(n)), "svr_timing_read")
    out = {}
    for i in range(n.value):
        nm = names.raw[i * L:(i + 1) * L].split(b"\0", 1)[0].decode()
        out[nm] = (float(ms[i]), int(cnt[i]))
    return out


def svr_graph_capture(scene, cams, n_cams, opts, ws, ws_bytes, rgba, grad_rgba, grad_grid, grad_sh,
                      extra, stream, graph_out):
    return load().svr_graph_capture(_ref(scene), cams, n_cams, _ref(opts), ws, ws_bytes, rgba,
                                    grad_rgba, grad_grid, grad_sh, _ref(extra), stream, graph_out)


def svr_graph_launch(graph, stream):
    return load().svr_graph_launch(graph, stream)


def svr_graph_destroy(graph):
    return load().svr_graph_destroy(graph)


def svr_grid_adjacency_scratch_bytes(n_voxels, n_grid):
    return load().svr_grid_adjacency_scratch_bytes(n_voxels, n_grid)


def svr_build_grid_adjacency(vox_grid, n_voxels, n_grid, adj_off, adj, scratch, scratch_bytes,
                             stream):
    return load().svr_build_grid_adjacency(vox_grid, n_voxels, n_grid, adj_off, adj, scratch,
                                           scratch_bytes, stream)


def svr_status_string(status):
    return load().svr_status_string(status).decode()


def svr_last_error():
    return load().svr_last_error().decode()


def svr_downsample(img_in, w_in, h_in, img_out, w_out, h_out, bg, stream):
    return load().svr_downsample(img_in, w_in, h_in, img_out, w_out, h_out, bg, stream)


def svr_downsample_bwd(grad_out, w_out, h_out, grad_in, w_in, h_in, bg, stream):
    return load().svr_downsample_bwd(grad_out, w_out, h_out, grad_in, w_in, h_in, bg, stream)


def svr_order_rank_scratch_bytes(n_voxels, max_level):
    return load().svr_order_rank_scratch_bytes(n_voxels, max_level)


def svr_build_order_ranks(octpath, n_voxels, max_level, rank, scratch, scratch_bytes, stream):
    return load().svr_build_order_ranks(octpath, n_voxels, max_level, rank, scratch,
                                        scratch_bytes, stream)


def svr_tsdf_fuse(grid_pos, n_grid, cams, n_cams, depth, rgba, min_alpha, trunc, tsdf, weight,
                  order, stream):
    return load().svr_tsdf_fuse(grid_pos, n_grid, cams, n_cams, depth, rgba, min_alpha, trunc,
                                tsdf, weight, order, stream)


def svr_marching_cubes(scene, field, weight, iso, max_triangles, tri_keys, tri_pos, n_triangles,
                       order, stream):
    return load().svr_marching_cubes(_ref(scene), field, weight, iso, max_triangles, tri_keys,
                                     tri_pos, n_triangles, order, stream)


def svr_morton_keys(pos, n, lo, extent, keys, values, stream):
    return load().svr_morton_keys(pos, n, lo, extent, keys, values, stream)


def svr_mesh_case_table(counts, verts):
    return load(with_torch=False).svr_mesh_case_table(counts, verts)
