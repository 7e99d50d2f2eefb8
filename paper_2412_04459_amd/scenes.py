"""Seeded synthetic scenes and cameras.

This module is shared by the GPU path, the tests and the benchmark, and holds
none of the renderer's arithmetic: it builds octree-leaf voxel sets (leaves
only, stored in arbitrary order, as in Sec. 3.1.1 "Sparse voxel grid"), the
shared corner grid points, corner raw densities, SH coefficients and pinhole
cameras.  Every array is plain numpy so either side can consume it.

Octree construction (the recipe the workloads are stated in):
  * nodes of the world cube (centre ``wc``, size ``ws``) at level l have size
    ``ws * 2**-l`` and integer index v in [0, 2**l)^3;
  * a node is subdivided while l < L_f for a surface f whose SDF at the node
    centre is within half the node diagonal plus ``kappa`` finest-level voxel
    sizes (so no leaf that the final rule keeps is ever missed);
  * at l == L_f a node is kept as a leaf iff |f(centre)| < kappa * size;
  * optional background shell: nodes whose centre radius lies in
    [bg_r0, bg_r1] are kept from level bg_l0 on, subdivided with probability
    bg_p until level bg_l1;
  * everything else is empty space and dropped.

Voxel octree paths are produced by the recursion itself: each subdivision
appends the child's 3-bit octant (x bit most significant) at the triplet of
its level, with level 1 in the top triplet of a 48-bit field (16 levels).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, List, Optional, Sequence

import numpy as np

MAX_LEVELS = 16


# ----------------------------------------------------------------------------
# surfaces (signed distance functions)
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class Sphere:
    center: Sequence[float]
    radius: float
    level: int

    def sdf(self, p: np.ndarray) -> np.ndarray:
        c = np.asarray(self.center, dtype=np.float64)
        return np.linalg.norm(p - c, axis=-1) - self.radius


@dataclasses.dataclass
class PlaneY:
    """Half-space y < y0 is solid; SDF = y - y0."""
    y0: float
    level: int

    def sdf(self, p: np.ndarray) -> np.ndarray:
        return p[..., 1] - self.y0


@dataclasses.dataclass
class Background:
    r0: float
    r1: float
    l0: int
    l1: int
    p: float


# ----------------------------------------------------------------------------
# scene container
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class Scene:
    world_center: np.ndarray      # (3,) f64
    world_size: float
    max_level: int
    ijk: np.ndarray               # (N,3) int64
    level: np.ndarray             # (N,) uint8
    center: np.ndarray            # (3,N) f32  SoA
    size: np.ndarray              # (N,) f32
    octpath: np.ndarray           # (N,) uint64
    vox_grid: np.ndarray          # (N,8) int32, corner c = 4dx+2dy+dz
    grid_pos: np.ndarray          # (M,3) f64 world position of grid points
    grid_raw: np.ndarray          # (M,) f32
    sh: np.ndarray                # (N,(D+1)^2,3) f32
    sh_degree: int

    @property
    def n_voxels(self) -> int:
        return int(self.size.shape[0])

    @property
    def n_grid(self) -> int:
        return int(self.grid_raw.shape[0])

    def subset(self, idx: np.ndarray) -> "Scene":
        """Voxel subset (keeps all grid points; unused ones are harmless)."""
        return dataclasses.replace(
            self, ijk=self.ijk[idx], level=self.level[idx],
            center=np.ascontiguousarray(self.center[:, idx]),
            size=self.size[idx], octpath=self.octpath[idx],
            vox_grid=np.ascontiguousarray(self.vox_grid[idx]),
            sh=np.ascontiguousarray(self.sh[idx]))


def _node_centers(wc, ws, lvl, ijk):
    s = ws * 2.0 ** (-lvl)
    return wc[None, :] - 0.5 * ws + s * (ijk.astype(np.float64) + 0.5), s


def build_octree(world_center, world_size, max_level, surfaces, kappa=1.0,
                 background: Optional[Background] = None,
                 rng: Optional[np.random.Generator] = None):
    """Return (ijk int64 (N,3), level uint8 (N,), octpath uint64 (N,))."""
    assert 1 <= max_level <= MAX_LEVELS
    wc = np.asarray(world_center, dtype=np.float64)
    ws = float(world_size)
    if rng is None:
        rng = np.random.default_rng(0)
    # level-1 nodes
    ijk = np.array([[x, y, z] for x in (0, 1) for y in (0, 1) for z in (0, 1)],
                   dtype=np.int64)
    path = ((ijk[:, 0] * 4 + ijk[:, 1] * 2 + ijk[:, 2]).astype(np.uint64)
            << np.uint64(3 * (MAX_LEVELS - 1)))
    out_ijk, out_lvl, out_path = [], [], []
    for lvl in range(1, max_level + 1):
        if ijk.shape[0] == 0:
            break
        c, s = _node_centers(wc, ws, lvl, ijk)
        keep = np.zeros(ijk.shape[0], dtype=bool)
        subdiv = np.zeros(ijk.shape[0], dtype=bool)
        for f in surfaces:
            d = np.abs(f.sdf(c))
            if lvl < f.level:
                subdiv |= d < (0.5 * math.sqrt(3.0) * s + kappa * ws * 2.0 ** (-f.level))
            elif lvl == f.level:
                keep |= d < kappa * s
        if background is not None:
            r = np.linalg.norm(c, axis=-1)
            inbg = (r >= background.r0) & (r <= background.r1)
            if lvl < background.l0:
                # coarse levels: descend everywhere the shell may be
                rc = np.linalg.norm(c, axis=-1)
                reach = 0.5 * math.sqrt(3.0) * s
                subdiv |= (rc + reach >= background.r0) & (rc - reach <= background.r1)
            elif lvl < background.l1:
                bg_sub = inbg & (rng.random(ijk.shape[0]) < background.p)
                subdiv |= bg_sub
                keep |= inbg & ~bg_sub
            elif lvl == background.l1:
                keep |= inbg
        keep &= ~subdiv
        if lvl == max_level:
            subdiv[:] = False
        out_ijk.append(ijk[keep])
        out_lvl.append(np.full(int(keep.sum()), lvl, dtype=np.uint8))
        out_path.append(path[keep])
        # children of subdivided nodes
        par = ijk[subdiv]
        ppath = path[subdiv]
        if par.shape[0] == 0:
            ijk = par
            continue
        kids = []
        kpath = []
        shift = np.uint64(3 * (MAX_LEVELS - (lvl + 1)))
        for bx in (0, 1):
            for by in (0, 1):
                for bz in (0, 1):
                    kids.append(par * 2 + np.array([bx, by, bz], dtype=np.int64))
                    kpath.append(ppath | (np.uint64(4 * bx + 2 * by + bz) << shift))
        ijk = np.concatenate(kids, axis=0)
        path = np.concatenate(kpath, axis=0)
    return (np.concatenate(out_ijk, 0), np.concatenate(out_lvl, 0),
            np.concatenate(out_path, 0))


def corner_grid(ijk, level, max_level):
    """Shared corner grid points.  Returns (vox_grid (N,8) int32, gkey (M,3) int64)
    with gkey the integer corner position at the finest level."""
    n = ijk.shape[0]
    sh = (max_level - level.astype(np.int64))
    base = ijk << sh[:, None]
    step = (np.int64(1) << sh)
    keys = np.empty((n, 8), dtype=np.int64)
    B = np.int64(max_level + 1)
    for c in range(8):
        dx, dy, dz = (c >> 2) & 1, (c >> 1) & 1, c & 1
        gx = base[:, 0] + dx * step
        gy = base[:, 1] + dy * step
        gz = base[:, 2] + dz * step
        keys[:, c] = (gx << (2 * B)) | (gy << B) | gz
    uniq, inv = np.unique(keys.reshape(-1), return_inverse=True)
    vox_grid = inv.reshape(n, 8).astype(np.int32)
    mask = (np.int64(1) << B) - 1
    g = np.stack([(uniq >> (2 * B)) & mask, (uniq >> B) & mask, uniq & mask], axis=1)
    return vox_grid, g


def make_scene(world_center, world_size, max_level, surfaces, *, kappa=1.0,
               background=None, sh_degree=0, sh_mode="rgb_uniform", sh_std=0.2,
               density_scale=-8.0, density_noise=0.1, opaque=False,
               seed=0) -> Scene:
    """Build a scene with the standard density recipe
    raw = density_scale * SDF(grid point) + N(0, density_noise)
    (SDF = signed min over surfaces).  ``opaque`` divides the SDF term by the
    squared finest voxel size, which gives an optical depth of order 10 per
    finest voxel inside surfaces (exercises early termination)."""
    ss = np.random.SeedSequence(seed).spawn(6)
    rng_geo, rng_den, rng_sh = (np.random.default_rng(s) for s in ss[:3])
    wc = np.asarray(world_center, dtype=np.float64)
    ws = float(world_size)
    ijk, lvl, path = build_octree(wc, ws, max_level, surfaces, kappa=kappa,
                                  background=background, rng=rng_geo)
    # shuffle: voxels are stored in arbitrary order
    perm = rng_geo.permutation(ijk.shape[0])
    ijk, lvl, path = ijk[perm], lvl[perm], path[perm]
    c, s = _node_centers(wc, ws, lvl.astype(np.float64)[:, None], ijk)
    s = s[:, 0]
    vox_grid, gint = corner_grid(ijk, lvl, max_level)
    gpos = wc[None, :] - 0.5 * ws + ws * gint.astype(np.float64) / float(2 ** max_level)
    if surfaces:
        sdf = np.min(np.stack([f.sdf(gpos) for f in surfaces], 0), axis=0)
    else:
        sdf = np.zeros(gpos.shape[0])
    if opaque:
        smin = ws * 2.0 ** (-max(f.level for f in surfaces))
        sdf = sdf / (smin * smin)
    raw = density_scale * sdf + rng_den.normal(0.0, density_noise, size=sdf.shape)
    nb = (sh_degree + 1) ** 2
    n = ijk.shape[0]
    if sh_mode == "rgb_uniform":
        # degree-0 band set so that the colour is U(0,1); higher bands N(0, std)
        sh = np.zeros((n, nb, 3), dtype=np.float64)
        y00 = 0.5 / math.sqrt(math.pi)
        sh[:, 0, :] = rng_sh.random((n, 3)) / y00
        if nb > 1:
            sh[:, 1:, :] = rng_sh.normal(0.0, sh_std, size=(n, nb - 1, 3))
    else:
        sh = rng_sh.normal(0.0, sh_std, size=(n, nb, 3))
    return Scene(world_center=wc, world_size=ws, max_level=max_level, ijk=ijk,
                 level=lvl.astype(np.uint8),
                 center=np.ascontiguousarray(c.T.astype(np.float32)),
                 size=s.astype(np.float32), octpath=path.astype(np.uint64),
                 vox_grid=vox_grid, grid_pos=gpos, grid_raw=raw.astype(np.float32),
                 sh=sh.astype(np.float32), sh_degree=sh_degree)


# ----------------------------------------------------------------------------
# cameras (OpenCV pinhole: x right, y down, z forward; w2c = [R | t])
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class Camera:
    W: int
    H: int
    fx: float
    fy: float
    cx: float
    cy: float
    w2c: np.ndarray   # (3,4) f64

    @property
    def n_pixels(self) -> int:
        return self.W * self.H

    def position(self) -> np.ndarray:
        R = self.w2c[:, :3]
        return -R.T @ self.w2c[:, 3]


def look_at(W, H, fov_x_deg, eye, target=(0.0, 0.0, 0.0), up=(0.0, 0.0, 1.0)) -> Camera:
    eye = np.asarray(eye, dtype=np.float64)
    fwd = np.asarray(target, dtype=np.float64) - eye
    fwd /= np.linalg.norm(fwd)
    upv = np.asarray(up, dtype=np.float64)
    if abs(float(np.dot(fwd, upv))) > 0.999:
        upv = np.array([0.0, 1.0, 0.0])
    right = np.cross(fwd, upv)
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    R = np.stack([right, down, fwd], 0)
    t = -R @ eye
    fx = 0.5 * W / math.tan(0.5 * math.radians(fov_x_deg))
    # round intrinsics to fp32 so that both sides see identical values
    f32 = lambda x: float(np.float32(x))
    w2c = np.concatenate([R, t[:, None]], 1).astype(np.float32).astype(np.float64)
    return Camera(W=int(W), H=int(H), fx=f32(fx), fy=f32(fx), cx=f32(0.5 * W),
                  cy=f32(0.5 * H), w2c=w2c)


def random_direction(rng) -> np.ndarray:
    v = rng.normal(size=3)
    return v / np.linalg.norm(v)


def orbit_cameras(n, W, H, fov_x_deg, radius, elevation_deg, phase0):
    cams = []
    el = math.radians(elevation_deg)
    for i in range(n):
        ph = phase0 + 2.0 * math.pi * i / n
        eye = radius * np.array([math.cos(el) * math.cos(ph), math.cos(el) * math.sin(ph),
                                 math.sin(el)])
        cams.append(look_at(W, H, fov_x_deg, eye))
    return cams


# ----------------------------------------------------------------------------
# the workloads
# ----------------------------------------------------------------------------
RESOLUTION_MIX = [(640, 480), (800, 600), (1024, 768), (1280, 720), (1297, 840),
                  (1600, 900), (1920, 1080)]


@dataclasses.dataclass
class Workload:
    name: str
    scene: Scene
    cameras: List[Camera]
    K: int
    t_stop: float = 1e-4
    activation: int = 0   # 0 explin, 1 softplus
    grad_seed: int = 0


def _sphere_shell_cfg(seed, n_spheres, lo, hi, rlo, rhi, level):
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(6)[0].generate_state(1)[0])
    cs = rng.uniform(lo, hi, size=(n_spheres, 3))
    rs = rng.uniform(rlo, rhi, size=n_spheres)
    return [Sphere(tuple(c), float(r), level) for c, r in zip(cs, rs)]


def sphere_shell_scene(opaque=False, seed=0) -> Scene:
    """~3.3k leaves: a level-6 shell of the sphere |p| = 0.5 inside [0,1]^3,
    kept where |SDF(centre)| < voxel size; SH degree 0, colour U(0,1)."""
    return make_scene((0.5, 0.5, 0.5), 1.0, 6, [Sphere((0, 0, 0), 0.5, 6)], kappa=1.0,
                      sh_degree=0, sh_mode="rgb_uniform", opaque=opaque, seed=seed)


def sphere_shell_camera(seed=0) -> Camera:
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(6)[3])
    d = random_direction(rng)
    return look_at(64, 64, 50.0, 2.0 * d)


def spheres_plane_scene(opaque=False, seed=1, kappa=0.68) -> Scene:
    """~185k leaves, max level 9: three level-9 sphere shells plus a level-8
    ground plane (off the dyadic grid), SH degree 3 ~ N(0, 0.2)."""
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(6)[0])
    cs = rng.uniform([-0.5, -0.2, -0.5], [0.5, 0.5, 0.5], size=(3, 3))
    rs = rng.uniform(0.15, 0.3, size=3)
    surf = [Sphere(tuple(c), float(r), 9) for c, r in zip(cs, rs)]
    surf.append(PlaneY(-0.5 + 0.37 / 256.0, 8))
    return make_scene((0.0, 0.0, 0.0), 2.0, 9, surf, kappa=kappa, sh_degree=3,
                      sh_mode="normal", sh_std=0.2, opaque=opaque, seed=seed)


def spheres_plane_camera(seed=1) -> Camera:
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(6)[3])
    d = random_direction(rng)
    d[2] = abs(d[2]) * 0.5 + 0.2
    d /= np.linalg.norm(d)
    return look_at(800, 800, 50.0, 2.5 * d)


def spheres_background_scene(seed=2, max_level=12, n_spheres=4, kappa=1.0, opaque=False) -> Scene:
    """~1.1M leaves in [-8,8]^3, max level 12: four level-12 sphere shells near
    the origin plus a sparse background shell (levels 4..7) for radius 2.5..8."""
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(6)[0])
    cs = rng.uniform(-0.7, 0.7, size=(n_spheres, 3))
    rs = rng.uniform(0.3, 0.5, size=n_spheres)
    surf = [Sphere(tuple(c), float(r), max_level) for c, r in zip(cs, rs)]
    bg = Background(2.5, 8.0, 4, 7, 0.5)
    return make_scene((0.0, 0.0, 0.0), 16.0, max_level, surf, kappa=kappa, background=bg,
                      sh_degree=3, sh_mode="normal", sh_std=0.2, opaque=opaque, seed=seed)


def orbit_cameras_1297x840(n=36, seed=2, W=1297, H=840) -> List[Camera]:
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(6)[3])
    phase = float(rng.uniform(0, 2 * math.pi))
    return orbit_cameras(n, W, H, 60.0, 2.0, 8.5, phase)


def large_shells_scene(seed=4, kappa=0.875, n_spheres=3) -> Scene:
    """~8M leaves in [-8,8]^3, max level 14: three level-14 sphere shells
    (radii U(0.25, 0.4)) plus the sparse background shell of levels 4..7 for
    radius 2.5..8; SH degree 3 ~ N(0, 0.2)."""
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(6)[0])
    cs = rng.uniform(-0.7, 0.7, size=(n_spheres, 3))
    rs = rng.uniform(0.25, 0.4, size=n_spheres)
    surf = [Sphere(tuple(c), float(r), 14) for c, r in zip(cs, rs)]
    bg = Background(2.5, 8.0, 4, 7, 0.5)
    return make_scene((0.0, 0.0, 0.0), 16.0, 14, surf, kappa=kappa, background=bg, sh_degree=3,
                      sh_mode="normal", sh_std=0.2, seed=seed)


def orbit_cameras_1080p(n=16, seed=4) -> List[Camera]:
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(6)[3])
    phase = float(rng.uniform(0, 2 * math.pi))
    return orbit_cameras(n, 1920, 1080, 60.0, 2.0, 8.5, phase)


def mixed_resolution_cameras(n=24, seed=3) -> List[Camera]:
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(6)[3])
    phase = float(rng.uniform(0, 2 * math.pi))
    res = [RESOLUTION_MIX[int(i)] for i in rng.integers(0, len(RESOLUTION_MIX), size=n)]
    cams = []
    for i, (W, H) in enumerate(res):
        ph = phase + 2.0 * math.pi * i / n
        el = math.radians(8.5)
        eye = 2.0 * np.array([math.cos(el) * math.cos(ph), math.cos(el) * math.sin(ph),
                              math.sin(el)])
        cams.append(look_at(W, H, 60.0, eye))
    return cams


def upstream_grads(n_pixels, seed) -> np.ndarray:
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(6)[4])
    return rng.normal(0.0, 1.0, size=(n_pixels, 4)).astype(np.float32)


def tiny_random_scene(seed, max_level=3, p_sub=0.5, sh_degree=1, density_std=1.0,
                      world_size=1.0) -> Scene:
    """Random non-overlapping octree in [0,1]^3 for brute-force checks: each
    node is subdivided with probability p_sub, kept otherwise (70%) or dropped."""
    rng = np.random.default_rng(seed)
    ijk = np.array([[x, y, z] for x in (0, 1) for y in (0, 1) for z in (0, 1)], np.int64)
    path = ((ijk[:, 0] * 4 + ijk[:, 1] * 2 + ijk[:, 2]).astype(np.uint64)
            << np.uint64(3 * (MAX_LEVELS - 1)))
    outs = []
    for lvl in range(1, max_level + 1):
        u = rng.random(ijk.shape[0])
        sub = (u < p_sub) if lvl < max_level else np.zeros_like(u, dtype=bool)
        keep = (~sub) & (rng.random(ijk.shape[0]) < 0.7)
        outs.append((ijk[keep], np.full(int(keep.sum()), lvl, np.uint8), path[keep]))
        par, pp = ijk[sub], path[sub]
        shift = np.uint64(3 * (MAX_LEVELS - (lvl + 1)))
        kids, kp = [], []
        for c in range(8):
            b = np.array([(c >> 2) & 1, (c >> 1) & 1, c & 1], np.int64)
            kids.append(par * 2 + b)
            kp.append(pp | (np.uint64(c) << shift))
        ijk = np.concatenate(kids, 0) if kids else ijk[:0]
        path = np.concatenate(kp, 0) if kp else path[:0]
    ijk = np.concatenate([o[0] for o in outs], 0)
    lvl = np.concatenate([o[1] for o in outs], 0)
    path = np.concatenate([o[2] for o in outs], 0)
    perm = rng.permutation(ijk.shape[0])
    ijk, lvl, path = ijk[perm], lvl[perm], path[perm]
    wc = np.full(3, 0.5 * world_size)
    c, s = _node_centers(wc, world_size, lvl.astype(np.float64)[:, None], ijk)
    vox_grid, gint = corner_grid(ijk, lvl, max_level)
    m = gint.shape[0]
    gpos = wc[None, :] - 0.5 * world_size + world_size * gint / float(2 ** max_level)
    raw = rng.normal(0.0, density_std, size=m) + 2.0
    nb = (sh_degree + 1) ** 2
    sh = rng.normal(0.0, 0.5, size=(ijk.shape[0], nb, 3))
    sh[:, 0, :] += 1.5
    return Scene(world_center=wc, world_size=world_size, max_level=max_level, ijk=ijk,
                 level=lvl, center=np.ascontiguousarray(c.T.astype(np.float32)),
                 size=s[:, 0].astype(np.float32), octpath=path, vox_grid=vox_grid,
                 grid_pos=gpos, grid_raw=raw.astype(np.float32), sh=sh.astype(np.float32),
                 sh_degree=sh_degree)


def scene_from_voxels(world_center, world_size, max_level, ijk, level, grid_raw=None,
                      sh=None, sh_degree=0) -> Scene:
    """Scene from an explicit voxel list (index + level).  ``grid_raw`` is a
    callable on grid-point world positions (M,3) or None (zeros); ``sh`` an
    (N,(D+1)^2,3) array or None (zeros)."""
    wc = np.asarray(world_center, dtype=np.float64)
    ws = float(world_size)
    ijk = np.asarray(ijk, dtype=np.int64).reshape(-1, 3)
    lvl = np.asarray(level, dtype=np.uint8).reshape(-1)
    path = np.zeros(ijk.shape[0], np.uint64)
    for n in range(ijk.shape[0]):
        # append octants coarsest first, as the recursion does
        p = 0
        for l in range(1, int(lvl[n]) + 1):
            sh_ = int(lvl[n]) - l
            oct_ = 4 * ((ijk[n, 0] >> sh_) & 1) + 2 * ((ijk[n, 1] >> sh_) & 1) + ((ijk[n, 2] >> sh_) & 1)
            p |= int(oct_) << (3 * (MAX_LEVELS - l))
        path[n] = p
    c, s = _node_centers(wc, ws, lvl.astype(np.float64)[:, None], ijk)
    vox_grid, gint = corner_grid(ijk, lvl, max_level)
    gpos = wc[None, :] - 0.5 * ws + ws * gint.astype(np.float64) / float(2 ** max_level)
    raw = np.zeros(gpos.shape[0]) if grid_raw is None else np.asarray(grid_raw(gpos), np.float64)
    nb = (sh_degree + 1) ** 2
    if sh is None:
        sh = np.zeros((ijk.shape[0], nb, 3))
    return Scene(world_center=wc, world_size=ws, max_level=max_level, ijk=ijk, level=lvl,
                 center=np.ascontiguousarray(c.T.astype(np.float32)),
                 size=s[:, 0].astype(np.float32), octpath=path, vox_grid=vox_grid,
                 grid_pos=gpos, grid_raw=raw.astype(np.float32),
                 sh=np.asarray(sh, np.float32).reshape(ijk.shape[0], nb, 3), sh_degree=sh_degree)


def sphere_depth_images(cams, spheres, hole_p=0.0, seed=0) -> List[np.ndarray]:
    """Synthetic depth images: per camera [H*W] float32, the distance along
    each pixel's unit ray (through the pixel centre) to the nearest of the
    spheres ((centre, radius) pairs), 0 where the ray misses them all or, with
    probability hole_p, at random pixels."""
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(6)[5])
    out = []
    for cam in cams:
        R = np.asarray(cam.w2c, np.float64)[:, :3]
        t = np.asarray(cam.w2c, np.float64)[:, 3]
        o = -R.T @ t
        u, v = np.meshgrid(np.arange(cam.W) + 0.5, np.arange(cam.H) + 0.5)
        dc = np.stack([(u - cam.cx) / cam.fx, (v - cam.cy) / cam.fy, np.ones_like(u)], -1)
        d = dc.reshape(-1, 3) @ R
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        best = np.full(d.shape[0], np.inf)
        for c, r in spheres:
            oc = o - np.asarray(c, np.float64)
            b = d @ oc
            disc = b * b - (oc @ oc - r * r)
            hit = disc >= 0
            tq = -b - np.sqrt(np.where(hit, disc, 0.0))
            hit &= tq > 0
            best = np.where(hit & (tq < best), tq, best)
        img = np.where(np.isfinite(best), best, 0.0)
        if hole_p > 0:
            img[rng.random(img.shape[0]) < hole_p] = 0.0
        out.append(img.astype(np.float32))
    return out


def camera_from_pose(W, H, fx, fy, cx, cy, R, t) -> Camera:
    w2c = np.concatenate([np.asarray(R, np.float64), np.asarray(t, np.float64)[:, None]], 1)
    f32 = lambda x: float(np.float32(x))
    return Camera(W=int(W), H=int(H), fx=f32(fx), fy=f32(fy), cx=f32(cx), cy=f32(cy),
                  w2c=w2c.astype(np.float32).astype(np.float64))


def workload(name: str, **kw) -> Workload:
    """Named workloads: "sphere_shell_3k", "sphere_shell_3k_opaque",
    "spheres_plane_184k", "orbit_1m_1297x840", "mixed_24cams_1m",
    "large_8m_16x1080p"."""
    if name == "sphere_shell_3k":
        return Workload(name, sphere_shell_scene(**kw), [sphere_shell_camera()], K=1, grad_seed=0)
    if name == "sphere_shell_3k_opaque":
        return Workload(name, sphere_shell_scene(opaque=True), [sphere_shell_camera()], K=1,
                        grad_seed=0)
    if name == "spheres_plane_184k":
        return Workload(name, spheres_plane_scene(**kw), [spheres_plane_camera()], K=1,
                        grad_seed=1)
    if name == "orbit_1m_1297x840":
        return Workload(name, spheres_background_scene(**kw), orbit_cameras_1297x840(), K=2,
                        grad_seed=2)
    if name == "large_8m_16x1080p":
        return Workload(name, large_shells_scene(**kw), orbit_cameras_1080p(), K=1, grad_seed=4)
    if name == "mixed_24cams_1m":
        return Workload(name, spheres_background_scene(**kw), mixed_resolution_cameras(), K=2,
                        grad_seed=3)
    raise KeyError(name)
