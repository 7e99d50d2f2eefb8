"""FP64 CPU oracle for the SVRaster sparse-voxel rasterizer (arXiv 2412.04459).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by
the CPU leg of the benchmark, never by the product path.  It shares no code
with the GPU library (see ``svr_oracle.c`` for what it computes and which
passage each function follows).

Parity pins (tests/test_oracle_*.py): explin/softplus closed forms and C1
continuity; trilinear partition of unity and corner reproduction; the uniform
voxel alpha = 1 - exp(-sigma l); SH orthonormality by quadrature, parity and
closed-form low bands; octree-path round trip against the scene recursion;
the permutation tables printed in Supp. B.2; agreement of the Morton rule
with entry-distance order on random octrees; FD checks of the adjoint.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "svr_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fopenmp", "-fPIC",
                               "-shared", "-fno-fast-math", "-ffp-contract=off", _SRC, "-o", tmp,
                               "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        _lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I64, I32, D = ctypes.c_int64, ctypes.c_int, ctypes.c_double
        _lib.oracle_render.argtypes = [I64, P, P, P, P, I64, P, I32, P, I32, D, I32, D, I64, P,
                                       P, P, P, P, P, P, I32, P, P, P, P, P, P, P, P, P, I32]
        _lib.oracle_render.restype = I32
        _lib.oracle_voxel_tiles.argtypes = [I64, P, P, P, I32, I32, D, D, P, P]
        _lib.oracle_downsample.argtypes = [P, I32, I32, P, I32, I32, P]
        _lib.oracle_downsample.restype = None
        _lib.oracle_downsample_adjoint.argtypes = [P, I32, I32, P, I32, I32, P]
        _lib.oracle_downsample_adjoint.restype = None
        _lib.oracle_voxel_tiles.restype = None
        _lib.oracle_tile_masks.argtypes = [P, I32, I32, D, P, P]
        _lib.oracle_tile_masks.restype = None
        _lib.oracle_keys.argtypes = [I64, P, P, P, P, I32, P, P, P]
        _lib.oracle_keys.restype = None
        _lib.oracle_to_octpath.argtypes = [I64, I64, I64, I32]
        _lib.oracle_to_octpath.restype = ctypes.c_uint64
        _lib.oracle_to_voxel_index.argtypes = [ctypes.c_uint64, I32, P]
        _lib.oracle_to_voxel_index.restype = None
        _lib.oracle_morton_order.argtypes = [ctypes.c_uint64, I32]
        _lib.oracle_morton_order.restype = ctypes.c_uint64
        _lib.oracle_child_rank.argtypes = [I32, I32]
        _lib.oracle_child_rank.restype = I32
        _lib.oracle_act.argtypes = [D, I32]
        _lib.oracle_act.restype = D
        _lib.oracle_act_grad.argtypes = [D, I32]
        _lib.oracle_act_grad.restype = D
        _lib.oracle_sh_basis.argtypes = [I32, P, P]
        _lib.oracle_sh_basis.restype = None
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def cam_array(cam) -> np.ndarray:
    """Camera as double[18]: W, H, fx, fy, cx, cy, then w2c (3x4 row-major)."""
    return np.concatenate([[cam.W, cam.H, cam.fx, cam.fy, cam.cx, cam.cy],
                           np.asarray(cam.w2c, np.float64).reshape(-1)]).astype(np.float64)


# --------------------------------------------------------------------------
# scalar helpers
# --------------------------------------------------------------------------
def act(x: float, kind: int = 0) -> float:
    return _load().oracle_act(float(x), int(kind))


def act_grad(x: float, kind: int = 0) -> float:
    return _load().oracle_act_grad(float(x), int(kind))


def sh_basis(degree: int, direction) -> np.ndarray:
    d = np.ascontiguousarray(direction, dtype=np.float64)
    out = np.zeros(16, np.float64)
    _load().oracle_sh_basis(int(degree), _p(d), _p(out))
    return out[: (degree + 1) ** 2]


def to_octpath(i: int, j: int, k: int, lv: int) -> int:
    return int(_load().oracle_to_octpath(int(i), int(j), int(k), int(lv)))


def to_voxel_index(path: int, lv: int):
    out = np.zeros(3, np.int64)
    _load().oracle_to_voxel_index(ctypes.c_uint64(int(path)), int(lv), _p(out))
    return tuple(int(x) for x in out)


def child_rank(s: int, t: int) -> int:
    return int(_load().oracle_child_rank(int(s), int(t)))


def morton_order(path: int, s: int) -> int:
    return int(_load().oracle_morton_order(ctypes.c_uint64(int(path)), int(s)))


# --------------------------------------------------------------------------
# rendering and gradients
# --------------------------------------------------------------------------
def render(scene, cam, K: int, t_stop: float = 1e-4, activation: int = 0, pixels=None,
           band: float = 1e-3, grad_rgba=None, max_seq: int = 0, nthreads: int = 0,
           train_stats: bool = False, depth_normal: bool = False, grad_depth=None,
           grad_normal=None) -> dict:
    """Brute-force FP64 render of the listed pixels (all when None).

    Returns dict(rgba, rgba_alt, flags, ncomp, nhit[, seq][, grad_grid, grad_sh]
    [, max_weight][, priority]).  ``grad_rgba`` (npix,4) gives dL/d rgba for
    L = sum <grad_rgba, rgba>.  ``train_stats`` adds the per-voxel maximum
    blending weight and (with grad_rgba) the subdivision priority.
    ``depth_normal`` adds the depth image [npix] and normal image [npix, 3];
    with grad_rgba, ``grad_depth`` [npix] and ``grad_normal`` [npix, 3] add
    <grad_depth, depth> + <grad_normal, normal> to L."""
    lib = _load()
    W, H = cam.W, cam.H
    if pixels is None:
        pixels = np.arange(W * H, dtype=np.int64)
    pixels = np.ascontiguousarray(pixels, dtype=np.int64)
    npix = pixels.shape[0]
    N = scene.n_voxels
    M = scene.n_grid
    # exact promotion of the scene parameters to double
    center = np.ascontiguousarray(scene.center, np.float64)
    size = np.ascontiguousarray(scene.size, np.float64)
    vg = np.ascontiguousarray(scene.vox_grid, np.int32)
    raw = np.ascontiguousarray(scene.grid_raw, np.float64)
    sh = np.ascontiguousarray(scene.sh, np.float64)
    ca = cam_array(cam)
    rgba = np.zeros((npix, 4), np.float64)
    alt = np.zeros((npix, 4), np.float64)
    flags = np.zeros(npix, np.uint8)
    ncomp = np.zeros(npix, np.int32)
    nhit = np.zeros(npix, np.int32)
    seq = np.full((npix, max_seq), -1, np.int32) if max_seq > 0 else None
    g = gg = gs = None
    if grad_rgba is not None:
        g = np.ascontiguousarray(grad_rgba, np.float64).reshape(npix, 4)
        gg = np.zeros(M, np.float64)
        gs = np.zeros(sh.shape, np.float64)
    mw = np.zeros(N, np.float64) if train_stats else None
    pr = np.zeros(N, np.float64) if (train_stats and g is not None) else None
    dep = np.zeros(npix, np.float64) if depth_normal else None
    nrm = np.zeros((npix, 3), np.float64) if depth_normal else None
    gd = None if (g is None or grad_depth is None) else \
        np.ascontiguousarray(grad_depth, np.float64).reshape(npix)
    gn = None if (g is None or grad_normal is None) else \
        np.ascontiguousarray(grad_normal, np.float64).reshape(npix, 3)
    lib.oracle_render(N, _p(center), _p(size), _p(vg), _p(raw), M, _p(sh), int(scene.sh_degree),
                      _p(ca), int(K), float(t_stop), int(activation), float(band), npix,
                      _p(pixels), _p(rgba), _p(alt), _p(flags), _p(ncomp), _p(nhit), _p(seq),
                      int(max_seq), _p(g), _p(gg), _p(gs), _p(mw), _p(pr), _p(dep), _p(nrm),
                      _p(gd), _p(gn), int(nthreads))
    out = dict(rgba=rgba, rgba_alt=alt, flags=flags, ncomp=ncomp, nhit=nhit, pixels=pixels)
    if mw is not None:
        out["max_weight"] = mw
    if pr is not None:
        out["priority"] = pr
    if dep is not None:
        out["depth"] = dep
        out["normal"] = nrm
    if seq is not None:
        out["seq"] = seq
    if g is not None:
        out["grad_grid"] = gg
        out["grad_sh"] = gs
    return out


# --------------------------------------------------------------------------
# projection, tile masks, keys
# --------------------------------------------------------------------------
Z_NEAR = 1e-4


def voxel_tiles(scene, cam, tile_w=16, tile_h=16, z_near=Z_NEAR, band=0.02):
    N = scene.n_voxels
    must = np.zeros((N, 4), np.int32)
    may = np.zeros((N, 4), np.int32)
    _load().oracle_voxel_tiles(N, _p(np.ascontiguousarray(scene.center, np.float64)),
                               _p(np.ascontiguousarray(scene.size, np.float64)),
                               _p(cam_array(cam)), int(tile_w), int(tile_h), float(z_near),
                               float(band), _p(must), _p(may))
    return must, may


def tile_masks(cam, tile_w=16, tile_h=16, rel_band=1e-6):
    ntx = (cam.W + tile_w - 1) // tile_w
    nty = (cam.H + tile_h - 1) // tile_h
    must = np.zeros(ntx * nty, np.uint8)
    may = np.zeros(ntx * nty, np.uint8)
    _load().oracle_tile_masks(_p(cam_array(cam)), int(tile_w), int(tile_h), float(rel_band),
                              _p(must), _p(may))
    return must, may


def keys(tile, vid, s, octpath, max_level):
    """(key_paper, key_compact, value) for (tile, voxel id, sign bits) triples."""
    tile = np.ascontiguousarray(tile, np.int64)
    vid = np.ascontiguousarray(vid, np.int64)
    s = np.ascontiguousarray(s, np.uint8)
    n = tile.shape[0]
    kp = np.zeros(n, np.uint64)
    kc = np.zeros(n, np.uint64)
    val = np.zeros(n, np.uint32)
    _load().oracle_keys(n, _p(tile), _p(vid), _p(s),
                        _p(np.ascontiguousarray(octpath, np.uint64)), int(max_level), _p(kp),
                        _p(kc), _p(val))
    return kp, kc, val


def _triples(rect, mask, ntx):
    """All (tile, vid, s) of voxel tile rectangles x tile sign masks."""
    ok = np.nonzero((rect[:, 0] <= rect[:, 1]) & (rect[:, 2] <= rect[:, 3]))[0]
    r = rect[ok].astype(np.int64)
    w = r[:, 1] - r[:, 0] + 1
    h = r[:, 3] - r[:, 2] + 1
    n = w * h
    total = int(n.sum())
    vid = np.repeat(ok.astype(np.int64), n)
    first = np.repeat(np.cumsum(n) - n, n)
    local = np.arange(total, dtype=np.int64) - first
    wr = np.repeat(w, n)
    tx = np.repeat(r[:, 0], n) + local % wr
    ty = np.repeat(r[:, 2], n) + local // wr
    tile = ty * ntx + tx
    m = mask[tile].astype(np.int64)
    tiles, vids, ss = [], [], []
    for s in range(8):
        sel = ((m >> s) & 1).astype(bool)
        tiles.append(tile[sel])
        vids.append(vid[sel])
        ss.append(np.full(int(sel.sum()), s, np.uint8))
    return np.concatenate(tiles), np.concatenate(vids), np.concatenate(ss)


def expected_entries(scene, cam, tile_w=16, tile_h=16, z_near=Z_NEAR, band=0.02,
                     rel_band=1e-6, tile_offset=0):
    """The duplicated (tile, voxel, s) list a tiled rasterizer must produce, as
    two bounds: ``must`` (every entry here has to be present) and ``may``
    (nothing outside it may be present).  Each is returned as sorted compact
    keys with values."""
    ntx = (cam.W + tile_w - 1) // tile_w
    r_must, r_may = voxel_tiles(scene, cam, tile_w, tile_h, z_near, band)
    m_must, m_may = tile_masks(cam, tile_w, tile_h, rel_band)
    out = {}
    for name, rect, mask in (("must", r_must, m_must), ("may", r_may, m_may)):
        t, v, s = _triples(rect, mask, ntx)
        kp, kc, val = keys(t + tile_offset, v, s, scene.octpath, scene.max_level)
        order = np.lexsort((val, kp))
        out[name] = (kc[order], val[order], kp[order])
    return out


# --------------------------------------------------------------------------
# anti-aliased downsampling and background (Sec. 3.1.2 "Anti-aliasing")
# --------------------------------------------------------------------------
def downsample(img, w_out: int, h_out: int, bg=None):
    """img [h_in, w_in, 4] (or [h_in * w_in, 4] with w_in given by shape) ->
    [h_out, w_out, 4]: separable tent filter of half-width n_in / n_out, then
    rgb += (1 - A) bg when bg is given."""
    img = np.ascontiguousarray(img, np.float64)
    h_in, w_in = img.shape[0], img.shape[1]
    out = np.zeros((h_out, w_out, 4), np.float64)
    b = None if bg is None else np.ascontiguousarray(bg, np.float64).reshape(3)
    _load().oracle_downsample(_p(img), int(w_in), int(h_in), _p(out), int(w_out), int(h_out), _p(b))
    return out


def downsample_adjoint(gout, w_in: int, h_in: int, bg=None):
    """D^T gout: gout [h_out, w_out, 4] -> [h_in, w_in, 4]."""
    gout = np.ascontiguousarray(gout, np.float64)
    h_out, w_out = gout.shape[0], gout.shape[1]
    gin = np.zeros((h_in, w_in, 4), np.float64)
    b = None if bg is None else np.ascontiguousarray(bg, np.float64).reshape(3)
    _load().oracle_downsample_adjoint(_p(gout), int(w_out), int(h_out), _p(gin), int(w_in),
                                      int(h_in), _p(b))
    return gin
