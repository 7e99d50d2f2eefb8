"""FP64 CPU oracle for sparse-voxel TSDF fusion and marching cubes
(Sec. 3.2.4 "Sparse-voxel TSDF Fusion and Marching Cubes").

TEST INFRASTRUCTURE ONLY: used by the tests and the smoke check, never by the
product path; it shares no code with the GPU library.

TSDF fusion (readings, the paper gives the method by reference only):
  for every grid point p and every camera with a depth image D (distance
  along the unit ray from the camera centre, the depth the renderer writes;
  values <= 0 mark pixels without depth): project p; when it lies in front of
  the camera and inside the image, take the pixel whose square holds the
  projection (centres at +0.5), and the signed distance along that ray
      sdf = D(pixel) - |p - o|.
  Observations with sdf >= -trunc are integrated as min(sdf / trunc, 1) with
  weight 1; the fused value is their mean (weight = their count).  Points
  never observed keep the value 1 and weight 0.  When the rendered opacity A
  is given with the depth (the renderer's depth is the composited sum
  sum_i T_i d_i), the distance is that sum divided by A where A >= min_alpha
  and A > 0 (the images are float32; the quotient is taken in FP64, and the
  points whose truncation decision lies within a relative 1e-6 of its
  threshold are reported as ties, where a float32 quotient may decide the
  other way); other pixels carry no depth.

Marching cubes over the voxels (one cell per voxel, its 8 corner grid
points; corner c = 4x + 2y + z):
  a corner is "above" when its value > iso.  The isosurface crosses every
  cell edge whose corners differ.  On each of the cell's 6 faces the crossing
  edges are joined in pairs: two crossings give one segment; four (above
  corners on a diagonal) give two segments, each cutting off one above
  corner.  Every segment is oriented so that the above corners it separates
  lie on its left seen from outside the cell; the oriented segments chain
  into closed loops, one polygon each, whose right-hand normal points towards
  increasing values.  A loop starts at its crossing edge with the smallest
  corner pair (8 a + b, a < b) and is cut into a fan of triangles from that
  vertex.  A vertex is identified by its edge's grid point pair (the smaller
  index first), so vertices shared by neighbouring cells merge; its position
  interpolates the corner positions linearly at the iso value.  Cells with a
  corner of weight 0 (when weights are given) produce nothing.
"""
from __future__ import annotations

import numpy as np

# corner c = 4x + 2y + z of the unit cell
_CORNER = np.array([[(c >> 2) & 1, (c >> 1) & 1, c & 1] for c in range(8)], dtype=np.float64)


def _cell_edges():
    return [(a, a | b) for b in (4, 2, 1) for a in range(8) if not a & b]


def _faces():
    """(outward normal, 4 corners around the face) for the 6 faces."""
    out = []
    for axis, bit in ((0, 4), (1, 2), (2, 1)):
        o1, o2 = [b for b in (4, 2, 1) if b != bit]
        for side in (0, 1):
            base = bit if side else 0
            ring = [base, base | o1, base | o1 | o2, base | o2]
            n = np.zeros(3)
            n[axis] = 1.0 if side else -1.0
            out.append((n, ring))
    return out


_EDGES = _cell_edges()
_FACES = _faces()


def cell_polygons(above):
    """Loops of the isosurface in one cell, as lists of corner pairs (a, b),
    a < b, in the orientation described in the module docstring.  `above`:
    8 booleans."""
    nxt = {}
    for n, ring in _FACES:
        cross = []
        for i in range(4):
            a, b = ring[i], ring[(i + 1) % 4]
            if above[a] != above[b]:
                cross.append(i)
        if not cross:
            continue
        segs = []  # (edge i, edge j, an above corner they cut off)
        if len(cross) == 2:
            ab = [q for q in ring if above[q]]
            segs.append((cross[0], cross[1], ab[0]))
        else:
            for j in range(4):
                if above[ring[j]]:
                    segs.append(((j - 1) % 4, j, ring[j]))
        for i, j, corner in segs:
            ei = tuple(sorted((ring[i], ring[(i + 1) % 4])))
            ej = tuple(sorted((ring[j], ring[(j + 1) % 4])))
            mi = 0.5 * (_CORNER[ei[0]] + _CORNER[ei[1]])
            mj = 0.5 * (_CORNER[ej[0]] + _CORNER[ej[1]])
            left = np.cross(n, mj - mi)
            if np.dot(left, _CORNER[corner] - mi) > 0:
                nxt[ei] = ej
            else:
                nxt[ej] = ei
    loops = []
    seen = set()
    for e0 in sorted(nxt, key=lambda e: 8 * e[0] + e[1]):
        if e0 in seen:
            continue
        loop = [e0]
        seen.add(e0)
        e = nxt[e0]
        while e != e0:
            if len(loop) > 12:
                raise RuntimeError("open isosurface loop")
            loop.append(e)
            seen.add(e)
            e = nxt[e]
        loops.append(loop)
    return loops


def cell_triangles(above):
    """Fan triangles (corner-pair triples) of one cell's loops."""
    tris = []
    for loop in cell_polygons(above):
        k = min(range(len(loop)), key=lambda i: 8 * loop[i][0] + loop[i][1])
        loop = loop[k:] + loop[:k]
        for i in range(1, len(loop) - 1):
            tris.append((loop[0], loop[i], loop[i + 1]))
    return tris


def marching_cubes(center, size, vox_grid, field, iso=0.0, weight=None):
    """Triangles of the iso-surface over the voxels.

    center [3][N] (or [N][3]), size [N], vox_grid [N][8], field [M] (values
    compared in float32, positions in float64), weight [M] or None.
    Returns (keys int64 [n][3][2] grid point pairs, pos float64 [n][3][3])."""
    center = np.asarray(center, np.float64)
    if center.shape[0] == 3 and center.ndim == 2 and center.shape[1] != 3:
        center = center.T
    size = np.asarray(size, np.float64)
    vox_grid = np.asarray(vox_grid, np.int64)
    f32 = np.asarray(field, np.float32)
    iso32 = np.float32(iso)
    keys, pos = [], []
    for v in range(vox_grid.shape[0]):
        g = vox_grid[v]
        if weight is not None and np.any(np.asarray(weight)[g] == 0):
            continue
        fv = f32[g]
        above = [bool(fv[c] > iso32) for c in range(8)]
        if all(above) or not any(above):
            continue
        corner_pos = center[v][None, :] + (_CORNER - 0.5) * size[v]
        for tri in cell_triangles(above):
            tk, tp = [], []
            for a, b in tri:
                fa, fb = float(fv[a]), float(fv[b])
                t = (float(iso32) - fa) / (fb - fa)
                tp.append(corner_pos[a] + t * (corner_pos[b] - corner_pos[a]))
                ga, gb = int(g[a]), int(g[b])
                tk.append((min(ga, gb), max(ga, gb)))
            keys.append(tk)
            pos.append(tp)
    return (np.asarray(keys, np.int64).reshape(-1, 3, 2), np.asarray(pos, np.float64).reshape(-1, 3, 3))


def tsdf_fuse(grid_pos, cams, depths, trunc, alphas=None, min_alpha=0.5, return_ties=False,
              tie_rel=1e-6):
    """Fused truncated signed distances of the grid points (values, weights).
    grid_pos [M][3]; depths / alphas: per camera [H*W] (alphas None: the
    depths are distances already; else the depths are composited sums and
    the distance is their FP64 quotient by the opacity where the opacity
    reaches min_alpha).  With ``return_ties`` also a mask of the points
    whose truncation decision (sdf >= -trunc) lies within ``tie_rel`` times
    the distance of its threshold in some camera: there a float32 quotient
    may decide the other way."""
    p = np.asarray(grid_pos, np.float64)
    M = p.shape[0]
    acc = np.zeros(M)
    w = np.zeros(M)
    ties = np.zeros(M, bool)
    for ci, (cam, D) in enumerate(zip(cams, depths)):
        if alphas is not None:
            # the opacity test compares two float32 values exactly
            A = np.asarray(alphas[ci], np.float32).reshape(-1)
            ok_a = (A >= np.float32(min_alpha)) & (A > 0)
            Dc = np.asarray(D, np.float32).reshape(-1).astype(np.float64)
            D = np.where(ok_a, Dc / np.where(ok_a, A, np.float32(1)).astype(np.float64), 0.0)
        D = np.asarray(D, np.float64).reshape(cam.H, cam.W)
        R = np.asarray(cam.w2c, np.float64)[:, :3]
        t = np.asarray(cam.w2c, np.float64)[:, 3]
        o = -R.T @ t
        pc = p @ R.T + t
        z = pc[:, 2]
        front = z > 0
        zs = np.where(front, z, 1.0)
        u = cam.fx * pc[:, 0] / zs + cam.cx
        v = cam.fy * pc[:, 1] / zs + cam.cy
        iu = np.floor(u)
        iv = np.floor(v)
        ok = front & (iu >= 0) & (iu < cam.W) & (iv >= 0) & (iv < cam.H)
        d = np.zeros(M)
        d[ok] = D[iv[ok].astype(np.int64), iu[ok].astype(np.int64)]
        ok &= d > 0
        sdf = d - np.linalg.norm(p - o[None, :], axis=1)
        ties |= ok & (np.abs(sdf + trunc) <= tie_rel * d)
        ok &= sdf >= -trunc
        acc[ok] += np.minimum(sdf[ok] / trunc, 1.0)
        w[ok] += 1.0
    val = np.where(w > 0, acc / np.maximum(w, 1.0), 1.0)
    if return_ties:
        return val, w, ties
    return val, w
