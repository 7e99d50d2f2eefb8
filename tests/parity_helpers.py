"""Checks shared by the GPU parity tests: the HIP path's outputs against the
FP64 oracle.

Bars:
- sorted (key, value) lists bit-exact: every entry's key equals the oracle's
  key of the same (tile, voxel, sign) triple, the list is strictly ascending,
  it holds every entry the oracle requires and nothing outside the oracle's
  tolerance band;
- RGBA within 1e-4 absolute per channel (either outcome of a flagged
  termination band is accepted);
- gradients within 1e-3 relative with an absolute floor of 1e-6 times the
  largest gradient of the tensor (the reading of "1e-3 relative" for entries
  that are sums of cancelling terms).
"""
import numpy as np

import oracle

RGBA_TOL = 1e-4
GRAD_REL = 1e-3
GRAD_FLOOR = 1e-6


def say(msg):
    print(msg, flush=True)


def check_rgba(gpu, ref, pixels=None, tol=RGBA_TOL):
    g = gpu if pixels is None else gpu[pixels]
    e1 = np.abs(g - ref["rgba"]).max(1)
    e2 = np.abs(g - ref["rgba_alt"]).max(1)
    err = np.minimum(e1, e2)
    worst = int(np.argmax(err))
    assert err.max() <= tol, "max |d rgba| = %.3g at sample %d (gpu %s, oracle %s)" % (
        err.max(), worst, g[worst], ref["rgba"][worst])
    return float(err.max())


def check_grad(g, r, name, rel=GRAD_REL, floor=GRAD_FLOOR):
    g = np.asarray(g, np.float64).reshape(-1)
    r = np.asarray(r, np.float64).reshape(-1)
    scale = np.abs(r).max()
    assert scale > 0
    tol = rel * np.abs(r) + floor * scale
    d = np.abs(g - r)
    bad = d > tol
    i = int(np.argmax(d - tol))
    assert not bad.any(), "%s: %d of %d entries off; worst %d gpu %.6g oracle %.6g (scale %.3g)" % (
        name, int(bad.sum()), r.size, i, g[i], r[i], scale)
    nz = np.abs(r) > floor * scale
    return float((d[nz] / np.abs(r[nz])).max()) if nz.any() else 0.0


def cpu_order_ranks(scene):
    """Rank of every (voxel, sign) pair in the oracle's within-tile key order."""
    n8 = 8 * scene.n_voxels
    vid = np.repeat(np.arange(scene.n_voxels, dtype=np.int64), 8)
    sgn = np.tile(np.arange(8, dtype=np.uint8), scene.n_voxels)
    _, kc, _ = oracle.keys(np.zeros(n8, np.int64), vid, sgn, scene.octpath, scene.max_level)
    order = np.argsort(kc, kind="stable")
    rank = np.empty(n8, np.int64)
    rank[order] = np.arange(n8)
    return rank


def key_low_bits(scene, ranks):
    return int(8 * scene.n_voxels - 1).bit_length() if ranks else 3 * scene.max_level + 3


def check_sorted_list(scene, cam, gk, gv, ranks, tile=16, tile_offset=0, rank_table=None):
    """One camera's block of the GPU's sorted list against the oracle: strictly
    ascending keys; each entry's value and, for its (tile, voxel, s), the
    oracle's key; those keys strictly ascending too (the list is in the
    paper's key order); the key's low bits are the order rank (ranks) or the
    compact key itself (no ranks); every required entry present and none
    outside the tolerance band.  ``tile_offset`` is the camera's first global
    tile id in a batched frame."""
    L = scene.max_level
    key_low = key_low_bits(scene, ranks)
    assert len(gk) > 0
    assert np.all(gk[1:] > gk[:-1])
    tid = (gk >> np.uint64(key_low)).astype(np.int64)
    vid = (gv & np.uint32((1 << 29) - 1)).astype(np.int64)
    sgn = (gv >> np.uint32(29)).astype(np.uint8)
    _, kc, val = oracle.keys(tid, vid, sgn, scene.octpath, L)
    assert np.array_equal(val, gv)
    assert np.all(kc[1:] > kc[:-1])
    if ranks:
        low = (gk & np.uint64((1 << key_low) - 1)).astype(np.int64)
        table = cpu_order_ranks(scene) if rank_table is None else rank_table
        assert np.array_equal(low, table[vid * 8 + sgn])
    else:
        assert np.array_equal(kc, gk)
    exp = oracle.expected_entries(scene, cam, tile_w=tile, tile_h=tile, tile_offset=tile_offset)
    must_k, _, _ = exp["must"]
    may_k, _, _ = exp["may"]
    assert np.all(np.isin(must_k, kc)), "missing %d required entries" % int((~np.isin(must_k, kc)).sum())
    assert np.all(np.isin(kc, may_k)), "%d entries outside the band" % int((~np.isin(kc, may_k)).sum())
    assert len(must_k) > 0
    return tid
