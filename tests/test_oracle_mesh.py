"""Pins of the mesh oracle (Sec. 3.2.4 "Sparse-voxel TSDF Fusion and Marching
Cubes"): the cell triangulation over all 256 corner cases, closed manifolds
with the right Euler characteristic for a sphere and a torus, exact planes
for linear fields, outward orientation, and the TSDF of a plane in closed
form."""
import itertools
import math

import numpy as np
import pytest

from oracle import mesh
from paper_2412_04459_amd import scenes as S


def _dense_grid(level, field_fn):
    """All voxels of `level` in [0, 1]^3 with grid values field_fn(positions)."""
    n = 1 << level
    g = np.stack(np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij"), -1).reshape(-1, 3)
    sc = S.scene_from_voxels((0.5, 0.5, 0.5), 1.0, level, g, np.full(len(g), level), grid_raw=field_fn)
    return sc


def _mesh_stats(keys):
    """(V, E, F, max and min count of triangles per mesh edge)."""
    vid = {}
    tri = []
    for t in keys:
        tri.append([vid.setdefault((int(k[0]), int(k[1])), len(vid)) for k in t])
    edges = {}
    for a, b, c in tri:
        for u, w in ((a, b), (b, c), (c, a)):
            e = (min(u, w), max(u, w))
            edges[e] = edges.get(e, 0) + 1
    cnt = np.array(list(edges.values()))
    return len(vid), len(edges), len(tri), int(cnt.max()), int(cnt.min())


def test_every_case_gives_closed_loops_over_its_crossing_edges():
    for case in range(256):
        above = [bool((case >> c) & 1) for c in range(8)]
        crossing = {(a, b) for a, b in mesh._EDGES if above[a] != above[b]}
        loops = mesh.cell_polygons(above)
        used = [e for loop in loops for e in loop]
        assert sorted(used) == sorted(crossing), case
        assert all(len(loop) >= 3 for loop in loops), case
        tris = mesh.cell_triangles(above)
        assert len(tris) == sum(len(loop) - 2 for loop in loops)


def test_single_corner_is_cut_off_by_one_triangle_facing_it():
    for c in range(8):
        above = [q == c for q in range(8)]
        tris = mesh.cell_triangles(above)
        assert len(tris) == 1
        # the triangle's normal (right-hand rule) points to the above corner
        cp = mesh._CORNER
        pts = [0.5 * (cp[a] + cp[b]) for a, b in tris[0]]
        nrm = np.cross(pts[1] - pts[0], pts[2] - pts[0])
        assert np.dot(nrm, cp[c] - np.mean(pts, 0)) > 0


@pytest.mark.parametrize("level", [3, 4])
def test_sphere_is_a_closed_outward_surface_of_euler_characteristic_two(level):
    ctr, rad = np.array([0.47, 0.52, 0.5]), 0.31
    sc = _dense_grid(level, lambda p: np.linalg.norm(p - ctr, axis=1) - rad)
    keys, pos = mesh.marching_cubes(sc.center, sc.size, sc.vox_grid, sc.grid_raw, 0.0)
    V, E, F, cmax, cmin = _mesh_stats(keys)
    assert cmax == 2 and cmin == 2  # every mesh edge borders exactly two triangles
    assert V - E + F == 2
    h = 1.0 / (1 << level)
    dist = np.abs(np.linalg.norm(pos - ctr, axis=2) - rad)
    assert dist.max() < 0.5 * h * h / rad + 1e-6
    nrm = np.cross(pos[:, 1] - pos[:, 0], pos[:, 2] - pos[:, 0])
    assert np.all(np.einsum("ij,ij->i", nrm, pos.mean(1) - ctr) > 0)


def test_torus_has_euler_characteristic_zero():
    R, r = 0.28, 0.11
    def f(p):
        q = p - 0.5
        return np.hypot(np.hypot(q[:, 0], q[:, 1]) - R, q[:, 2]) - r
    sc = _dense_grid(5, f)
    keys, _ = mesh.marching_cubes(sc.center, sc.size, sc.vox_grid, sc.grid_raw, 0.0)
    V, E, F, cmax, cmin = _mesh_stats(keys)
    assert cmax == 2 and cmin == 2
    assert V - E + F == 0


def test_linear_field_gives_the_exact_plane_and_area():
    nrm = np.array([0.0, 0.0, 1.0])
    sc = _dense_grid(3, lambda p: p @ nrm - 0.3)
    keys, pos = mesh.marching_cubes(sc.center, sc.size, sc.vox_grid, sc.grid_raw, 0.0)
    assert np.abs(pos @ nrm - 0.3).max() < 1e-7
    area = 0.5 * np.linalg.norm(np.cross(pos[:, 1] - pos[:, 0], pos[:, 2] - pos[:, 0]), axis=1).sum()
    assert abs(area - 1.0) < 1e-6
    # oblique plane: still exact (trilinear fields that are linear)
    nrm2 = np.array([0.3, -0.5, 0.81])
    nrm2 /= np.linalg.norm(nrm2)
    sc = _dense_grid(3, lambda p: p @ nrm2 - 0.1)
    _, pos = mesh.marching_cubes(sc.center, sc.size, sc.vox_grid, sc.grid_raw, 0.0)
    assert np.abs(pos @ nrm2 - 0.1).max() < 1e-6


def test_weight_zero_cells_are_skipped():
    ctr, rad = np.array([0.5, 0.5, 0.5]), 0.3
    sc = _dense_grid(3, lambda p: np.linalg.norm(p - ctr, axis=1) - rad)
    w = np.ones(sc.n_grid)
    keys_all, _ = mesh.marching_cubes(sc.center, sc.size, sc.vox_grid, sc.grid_raw, 0.0)
    w[sc.vox_grid[:, 0]] = 0.0
    keys_w, _ = mesh.marching_cubes(sc.center, sc.size, sc.vox_grid, sc.grid_raw, 0.0, weight=w)
    assert len(keys_w) < len(keys_all)


def test_tsdf_of_a_plane_along_pixel_rays_in_closed_form():
    # a camera at height 2 looking down at the plane z = 0
    cam = S.look_at(32, 24, 70.0, [0.0, 0.0, 2.0], target=(0.0, 0.0, 0.0), up=(0.0, 1.0, 0.0))
    R = cam.w2c[:, :3]
    o = cam.position()
    uu, vv = np.meshgrid(np.arange(cam.W) + 0.5, np.arange(cam.H) + 0.5)
    d_cam = np.stack([(uu - cam.cx) / cam.fx, (vv - cam.cy) / cam.fy, np.ones_like(uu)], -1)
    d = d_cam @ R  # rows: R^T d_cam
    d /= np.linalg.norm(d, axis=-1, keepdims=True)
    depth = -o[2] / d[..., 2]  # ray distance to z = 0
    # grid points on the centre rays of a few pixels, at several distances
    rng = np.random.default_rng(0)
    pix = rng.integers(0, cam.W * cam.H, 40)
    s = rng.uniform(1.5, 2.8, 40)
    dirs = d.reshape(-1, 3)[pix]
    pts = o[None, :] + s[:, None] * dirs
    trunc = 0.2
    val, w = mesh.tsdf_fuse(pts, [cam], [depth], trunc)
    sdf = depth.reshape(-1)[pix] - s
    use = sdf >= -trunc
    assert np.all(w[use] == 1) and np.all(w[~use] == 0)
    assert np.allclose(val[use], np.minimum(sdf[use] / trunc, 1.0), atol=1e-9)
    assert np.all(val[~use] == 1.0)
    # a second identical view averages to the same values, weight 2
    val2, w2 = mesh.tsdf_fuse(pts, [cam, cam], [depth, depth], trunc)
    assert np.allclose(val2[use], val[use]) and np.all(w2[use] == 2)
    # pixels without depth are not integrated
    val3, w3 = mesh.tsdf_fuse(pts, [cam], [np.zeros_like(depth)], trunc)
    assert np.all(w3 == 0) and np.all(val3 == 1.0)
    # the renderer's composited depth with opacity A: the sum D A divided by
    # A where A >= min_alpha gives the same distances; below it, no depth
    A = rng.uniform(0.55, 1.0, size=depth.shape).astype(np.float32)
    comp = (depth * A).astype(np.float32)
    val4, w4 = mesh.tsdf_fuse(pts, [cam], [comp], trunc, alphas=[A], min_alpha=0.5)
    assert np.array_equal(w4, w)
    assert np.allclose(val4, val, atol=2e-6 / trunc)
    val5, w5 = mesh.tsdf_fuse(pts, [cam], [comp], trunc, alphas=[A * 0.5], min_alpha=0.5)
    assert np.all(w5 == 0) and np.all(val5 == 1.0)
