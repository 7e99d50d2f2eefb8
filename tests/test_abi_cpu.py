"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function include/svraster.h declares, and rejects bad arguments before
touching the device."""
import ctypes
import os

import numpy as np
import pytest

from paper_2412_04459_amd import _abi


def _lib():
    if not os.path.exists(_abi.LIB_PATH):
        pytest.skip("libsvraster.so not built")
    return _abi.load(with_torch=False)


def test_exports_every_declared_function():
    lib = _lib()
    names = _abi.header_functions()
    assert "svr_preprocess" in names and "svr_render_bwd" in names
    for n in names:
        assert hasattr(lib, n), n
    assert set(_abi._SIGS) == set(names)


def _host_args(N=1000, W=64, H=48, K=1, cap=4096):
    sc = _abi.svr_scene()
    sc.n_voxels = N
    sc.n_grid = 2 * N
    fake = 0x10000  # never dereferenced by the host-side checks
    for f in ("center", "size", "octpath", "vox_grid", "grid_raw", "sh"):
        setattr(sc, f, fake)
    sc.sh_degree = 3
    sc.max_level = 12
    cams = (_abi.svr_camera * 2)()
    for c in cams:
        c.width, c.height = W, H
        c.fx = c.fy = 50.0
        c.cx, c.cy = W / 2, H / 2
        for k, v in enumerate([1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 3]):
            c.w2c[k] = v
    o = _abi.svr_opts()
    o.K = K
    o.t_stop = 1e-4
    o.activation = 0
    o.entry_capacity = cap
    return sc, cams, o


def test_workspace_size_is_monotone_in_capacity_and_cameras():
    _lib()
    sc, cams, o = _host_args()
    a = _abi.svr_workspace_bytes(sc, cams, 1, o)
    assert a > 0
    o.entry_capacity = 8192
    b = _abi.svr_workspace_bytes(sc, cams, 1, o)
    assert b >= a + 4096 * 24
    c = _abi.svr_workspace_bytes(sc, cams, 2, o)
    assert c > b


@pytest.mark.parametrize("field,value", [("K", 0), ("K", 9), ("activation", 7),
                                         ("entry_capacity", 1 << 30), ("t_stop", -1.0),
                                         ("tile", 12), ("tile", 64), ("persistent", -1),
                                         ("accumulate", 2)])
def test_invalid_options_are_rejected(field, value):
    _lib()
    sc, cams, o = _host_args()
    setattr(o, field, value)
    assert _abi.svr_workspace_bytes(sc, cams, 1, o) == 0
    rc = _abi.svr_preprocess(sc, cams, 1, o, ctypes.c_void_p(0x100000), 1 << 30, None, None)
    assert rc == _abi.SVR_E_INVALID
    assert len(_abi.svr_last_error()) > 0


@pytest.mark.parametrize("field,value", [("n_voxels", 1 << 29), ("sh_degree", 4), ("max_level", 0),
                                         ("max_level", 17), ("n_voxels", -1)])
def test_invalid_scene_is_rejected(field, value):
    _lib()
    sc, cams, o = _host_args()
    setattr(sc, field, value)
    assert _abi.svr_workspace_bytes(sc, cams, 1, o) == 0
    for fn in (lambda: _abi.svr_sort(sc, cams, 1, o, ctypes.c_void_p(0x100000), 1 << 30, -1, None),
               lambda: _abi.svr_render_fwd(sc, cams, 1, o, ctypes.c_void_p(0x100000), 1 << 30,
                                           ctypes.c_void_p(0x1000), None, None)):
        assert fn() == _abi.SVR_E_INVALID


def test_camera_limits_and_workspace_checks():
    _lib()
    sc, cams, o = _host_args()
    assert _abi.svr_workspace_bytes(sc, cams, 0, o) == 0
    assert _abi.svr_workspace_bytes(sc, cams, 33, o) == 0
    cams[0].width = 0
    assert _abi.svr_workspace_bytes(sc, cams, 1, o) == 0
    cams[0].width = 64
    need = _abi.svr_workspace_bytes(sc, cams, 1, o)
    rc = _abi.svr_preprocess(sc, cams, 1, o, ctypes.c_void_p(0x100000), need - 1, None, None)
    assert rc == _abi.SVR_E_WORKSPACE
    rc = _abi.svr_preprocess(sc, cams, 1, o, ctypes.c_void_p(0x100010), need, None, None)
    assert rc == _abi.SVR_E_INVALID  # misaligned
    rc = _abi.svr_preprocess(sc, cams, 1, o, None, need, None, None)
    assert rc == _abi.SVR_E_INVALID
    # a 4096^2 frame at max_level 16 needs 16 + 48 + 3 key bits
    sc.max_level = 16
    cams[0].width = cams[0].height = 4096
    assert _abi.svr_workspace_bytes(sc, cams, 1, o) == 0


def test_sort_entry_point_checks():
    _lib()
    assert _abi.svr_radix_sort_scratch_bytes(1000, 52) > 0
    assert _abi.svr_radix_sort_scratch_bytes(-1, 52) == 0
    assert _abi.svr_radix_sort_pairs(None, None, None, None, 10, 65, None, 0, None) == _abi.SVR_E_INVALID
    assert _abi.svr_radix_sort_pairs(None, None, None, None, 0, 32, None, 0, None) == _abi.SVR_OK
    assert _abi.svr_status_string(_abi.SVR_E_CAPACITY) == "entry capacity exceeded"


def test_graph_entry_points_check_arguments():
    _lib()
    sc, cams, o = _host_args()
    h = ctypes.c_void_p(0)
    # the NULL stream cannot be captured
    rc = _abi.svr_graph_capture(sc, cams, 1, o, ctypes.c_void_p(0x100000), 1 << 30, None, None,
                                None, None, None, None, ctypes.byref(h))
    assert rc == _abi.SVR_E_INVALID and h.value is None
    assert _abi.svr_graph_launch(None, None) == _abi.SVR_E_INVALID
    assert _abi.svr_graph_destroy(None) == _abi.SVR_OK


@pytest.mark.parametrize("tile", [8, 16, 32])
def test_workspace_shrinks_with_larger_tiles(tile):
    _lib()
    sc, cams, o = _host_args(W=640, H=480)
    o.tile = tile
    assert _abi.svr_workspace_bytes(sc, cams, 1, o) > 0


def test_workspace_parts_sum_to_total():
    _lib()
    sc, cams, o = _host_args(N=5000, W=100, H=60, cap=70000)
    for n_cams in (1, 2):
        parts = _abi.svr_workspace_parts(sc, cams, n_cams, o)
        assert list(parts) == list(_abi.WS_PART_NAMES)
        assert sum(parts.values()) == _abi.svr_workspace_bytes(sc, cams, n_cams, o)
        # keys (8 B) + values (4 B), two buffers, 256-byte aligned each
        assert 24 * 70000 <= parts["keys_values_x2"] <= 24 * 70000 + 4 * 256
        # count, rect (4 + 8 B) and a 64-byte record per (voxel, camera)
        nv = 5000 * n_cams
        assert 76 * nv <= parts["per_voxel_camera_records"] <= 76 * nv + 3 * 256
        # one 8-byte partial entry total per 256 (voxel, camera) pairs
        assert 8 * ((nv + 255) // 256) <= parts["scan_partials"] <= 8 * ((nv + 255) // 256) + 256
        # 8 B per pixel, plus two 16 B checkpoints (colour, depth and normal)
        # per pixel of a 16x16 tile for each possible backward chunk
        # (capacity / 256 + 1)
        ck = 2 * (70000 // 256 + 1) * 256 * 16
        assert 8 * 6000 * n_cams + ck <= parts["per_pixel_state"] <= 8 * 6000 * n_cams + ck + 768
    with pytest.raises(ValueError):
        o.K = 0
        _abi.svr_workspace_parts(sc, cams, 1, o)


def test_downsample_rejects_bad_sizes():
    _lib()
    p = ctypes.c_void_p(0x100000)
    for (wi, hi, wo, ho) in ((10, 10, 11, 5), (10, 10, 0, 5), (10, 10, 5, 11), (70000, 10, 5, 5)):
        assert _abi.svr_downsample(p, wi, hi, p, wo, ho, None, None) == _abi.SVR_E_INVALID
        assert _abi.svr_downsample_bwd(p, wo, ho, p, wi, hi, None, None) == _abi.SVR_E_INVALID
    assert _abi.svr_downsample(None, 10, 10, p, 5, 5, None, None) == _abi.SVR_E_INVALID


def test_mesh_case_table_matches_the_oracle_cell_rule():
    """The library's compile-time cell table against the oracle's face-traced
    loops (Sec. 3.2.4 marching cubes), case by case and triangle by triangle."""
    _lib()
    from oracle import mesh as om
    counts = (ctypes.c_uint8 * 256)()
    verts = (ctypes.c_uint8 * (256 * 36))()
    assert _abi.svr_mesh_case_table(counts, verts) == _abi.SVR_OK
    v = np.frombuffer(verts, np.uint8).reshape(256, 36)
    for case in range(256):
        above = [bool((case >> c) & 1) for c in range(8)]
        tris = om.cell_triangles(above) if 0 < case < 255 else []
        assert counts[case] == len(tris), case
        got = [tuple((int(v[case, 3 * t + j]) >> 3, int(v[case, 3 * t + j]) & 7) for j in range(3))
               for t in range(len(tris))]
        assert got == [tuple(tuple(e) for e in tri) for tri in tris], case
    assert max(counts) <= 12
    assert _abi.svr_mesh_case_table(None, verts) == _abi.SVR_E_INVALID


def test_mesh_entry_points_check_arguments():
    _lib()
    sc, cams, _ = _host_args()
    p = ctypes.c_void_p(0x100000)
    # TSDF fusion: sizes, truncation, opacity threshold, cameras, null arrays
    assert _abi.svr_tsdf_fuse(p, -1, cams, 1, p, None, 0.5, 0.1, p, p, None, None) == _abi.SVR_E_INVALID
    assert _abi.svr_tsdf_fuse(p, 10, cams, 1, p, None, 0.5, 0.0, p, p, None, None) == _abi.SVR_E_INVALID
    assert _abi.svr_tsdf_fuse(p, 10, cams, 1, p, None, float("nan"), 0.1, p, p, None,
                              None) == _abi.SVR_E_INVALID
    assert _abi.svr_tsdf_fuse(p, 10, cams, 0, p, None, 0.5, 0.1, p, p, None, None) == _abi.SVR_E_INVALID
    assert _abi.svr_tsdf_fuse(None, 10, cams, 1, p, None, 0.5, 0.1, p, p, None,
                              None) == _abi.SVR_E_INVALID
    assert _abi.svr_tsdf_fuse(None, 0, cams, 1, None, None, 0.5, 0.1, None, None, None,
                              None) == _abi.SVR_OK
    # marching cubes: counter, arrays, iso, sizes
    assert _abi.svr_marching_cubes(sc, p, None, 0.0, 10, p, p, None, None, None) == _abi.SVR_E_INVALID
    assert _abi.svr_marching_cubes(sc, p, None, 0.0, 10, None, p, p, None, None) == _abi.SVR_E_INVALID
    assert _abi.svr_marching_cubes(sc, p, None, float("inf"), 10, p, p, p, None,
                                   None) == _abi.SVR_E_INVALID
    assert _abi.svr_marching_cubes(sc, p, None, 0.0, -1, p, p, p, None, None) == _abi.SVR_E_INVALID
    assert _abi.svr_marching_cubes(sc, None, None, 0.0, 10, p, p, p, None, None) == _abi.SVR_E_INVALID
    sc.n_grid = 1 << 31
    assert _abi.svr_marching_cubes(sc, p, None, 0.0, 10, p, p, p, None, None) == _abi.SVR_E_INVALID


def test_tsdf_fusion_checks_every_camera_beyond_one_group():
    """More cameras than one launch takes: each is still validated, and the
    error names its index in the caller's array."""
    _lib()
    n = 40
    cams = (_abi.svr_camera * n)()
    for c in cams:
        c.width, c.height = 32, 24
        c.fx = c.fy = 30.0
        c.cx, c.cy = 16.0, 12.0
        for k, v in enumerate([1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 3]):
            c.w2c[k] = v
    p = ctypes.c_void_p(0x100000)
    cams[35].fx = -1.0
    assert _abi.svr_tsdf_fuse(p, 10, cams, n, p, None, 0.5, 0.1, p, p, None, None) == _abi.SVR_E_INVALID
    assert "camera 35" in _abi.svr_last_error()



def test_morton_keys_check_arguments():
    _lib()
    p = ctypes.c_void_p(0x100000)
    lo = (ctypes.c_float * 3)(0.0, 0.0, 0.0)
    bad = (ctypes.c_float * 3)(0.0, float("nan"), 0.0)
    assert _abi.svr_morton_keys(p, -1, lo, 1.0, p, p, None) == _abi.SVR_E_INVALID
    assert _abi.svr_morton_keys(p, 10, bad, 1.0, p, p, None) == _abi.SVR_E_INVALID
    assert _abi.svr_morton_keys(p, 10, lo, 0.0, p, p, None) == _abi.SVR_E_INVALID
    assert _abi.svr_morton_keys(None, 10, lo, 1.0, p, p, None) == _abi.SVR_E_INVALID
    assert _abi.svr_morton_keys(None, 0, lo, 1.0, None, None, None) == _abi.SVR_OK


def test_zcurve_relabel_is_a_relabeling_in_octree_path_order():
    from paper_2412_04459_amd import scenes as S
    from paper_2412_04459_amd.render import zcurve_relabel
    sc = S.tiny_random_scene(5, max_level=4, sh_degree=1)
    rs, order = zcurve_relabel(sc)
    assert np.all(rs.octpath[1:] > rs.octpath[:-1])
    assert np.array_equal(np.sort(order), np.arange(sc.n_voxels))
    assert np.array_equal(rs.center, sc.center[:, order])
    assert np.array_equal(rs.sh, sc.sh[order])
    # grid points relabeled along the Z-curve: every voxel keeps its corner
    # positions and densities, and the stored positions follow the curve
    assert np.array_equal(rs.grid_raw[rs.vox_grid], sc.grid_raw[sc.vox_grid[order]])
    assert np.array_equal(rs.grid_pos[rs.vox_grid], sc.grid_pos[sc.vox_grid[order]])
    assert np.array_equal(np.sort(rs.grid_raw), np.sort(sc.grid_raw))
    L = sc.max_level
    lo = np.asarray(sc.world_center) - 0.5 * sc.world_size
    g = np.rint((rs.grid_pos - lo) / (sc.world_size / 2 ** L)).astype(np.int64)

    def morton(p):
        code = 0
        for b in range(L, -1, -1):
            for a in range(3):
                code = (code << 1) | ((int(p[a]) >> b) & 1)
        return code

    codes = [morton(p) for p in g]
    assert all(codes[i] < codes[i + 1] for i in range(len(codes) - 1))
    rv, _ = zcurve_relabel(sc, grid_points=False)
    assert np.array_equal(rv.vox_grid, sc.vox_grid[order])
    assert np.array_equal(rv.grid_raw, sc.grid_raw)
