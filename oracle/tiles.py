"""Tile-level integer rules, written plainly with NumPy stable sorts.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper partitions the grid into tiles (Sect. 3.1) and moves particles that
leave a tile to its neighbour (the particle-communication rows of Table 1);
it keeps particles unsorted inside a tile.  The GPU path stores, per tile,
positions relative to the tile centre.  These functions state what that
layout must hold, so that the GPU's integer work (tile and cell keys,
permutations, migration counts) can be checked bit-exactly:

* binning: tile t_d = floor(x_d / T_d); local x = fl_p(x - centre) with the
  centre t_d T_d + T_d/2 (the subtraction is exact in FP64); a value that
  rounds to +T_d/2 belongs to the next tile at -T_d/2 (with walls in x,
  except across the wall at x = n0: it stays just below the face).  Order
  inside a tile is the input order (stable).
* migration after a push: a particle whose local coordinate left
  [-T/2, T/2) moves to the neighbour tile (offset delta in {-1,0,1}^D) with
  local x - delta T (exact).  New order inside tile r: its stayers in their
  old order, then, for each direction code in increasing order, the
  particles arriving from tile r - delta in their old order.  Direction
  code: sum_d (delta_d + 1) 3^d.
* cell key: sum_d (floor(x_loc_d) + T_d/2) * prod_{d'<d} T_d' (x fastest);
  the cell sort is a stable sort by this key inside each tile.
* near-face flag: some local coordinate lies within 2 units in the last
  place of the storage precision at the tile half-width, 2 ulp_p(T_d/2), of
  an integer (a cell face).  Every coordinate of the tile is at most T_d/2 in
  size, so this holds every particle within 1 ulp of its own value of a
  face.
* migration counts: for every tile and direction code, the particles that
  were in the tile before the step and are in the neighbour at that offset
  after it (the centre code: those that stayed).
"""
from __future__ import annotations

import numpy as np


def tile_grid(n, T, D):
    return [n[d] // T[d] if d < D else 1 for d in range(3)]


def tile_linear(tc, nt):
    return tc[0] + nt[0] * (tc[1] + nt[1] * tc[2])


def bin_global(x, n, T, D, dtype, walls=False):
    """Bin global FP64 positions (D, np) into tiles.

    Returns (tile_id (np,), x_loc (D, np) in dtype, order) where ``order`` is
    the stable permutation that groups particles by tile id.  A local
    coordinate that rounds onto the upper tile face moves to the next tile at
    -T/2; with walls in x, one that would cross the wall at x = n0 stays in
    the last tile just below the face instead."""
    x = np.asarray(x, dtype=np.float64)
    npart = x.shape[1]
    nt = tile_grid(n, T, D)
    tc = np.zeros((3, npart), dtype=np.int64)
    xl = np.zeros((D, npart), dtype=dtype)
    for d in range(D):
        t = np.floor(x[d] / T[d]).astype(np.int64)
        t = np.clip(t, 0, nt[d] - 1)
        centre = t * T[d] + T[d] // 2
        loc = (x[d] - centre.astype(np.float64)).astype(dtype)
        half = dtype(T[d] // 2)
        up = loc >= half
        stay = up & (d == 0) & walls & (t == nt[d] - 1)
        move = up & ~stay
        t = np.where(move, (t + 1) % nt[d], t)
        loc = np.where(move, -half, loc).astype(dtype)
        loc = np.where(stay, np.nextafter(half, dtype(0)), loc).astype(dtype)
        tc[d] = t
        xl[d] = loc
    tid = tile_linear(tc, nt)
    order = np.argsort(tid, kind="stable")
    return tid, xl, order


def cell_key(xl, T, D):
    """Cell index inside the tile, x fastest, from centre-relative positions."""
    key = np.zeros(xl.shape[1], dtype=np.int64)
    stride = 1
    for d in range(D):
        c = np.floor(xl[d].astype(np.float64)).astype(np.int64) + T[d] // 2
        key += c * stride
        stride *= T[d]
    return key


def near_face_band(T, D, dtype):
    """Per dimension: 2 ulps of the storage precision at T_d / 2."""
    return [2.0 * float(np.spacing(dtype(T[d] // 2))) for d in range(D)]


def near_face(xl, D, T):
    """True where some local coordinate lies within the near-face band of an
    integer (distances computed exactly in FP64)."""
    band = near_face_band(T, D, xl.dtype.type)
    flag = np.zeros(xl.shape[1], dtype=bool)
    for d in range(D):
        v = xl[d].astype(np.float64)
        flag |= np.abs(v - np.round(v)) <= band[d]
    return flag


def direction(xl, T, D):
    """Offset code sum (delta_d + 1) 3^d of the tile a particle moved to."""
    code = np.zeros(xl.shape[1], dtype=np.int64)
    delta = np.zeros((3, xl.shape[1]), dtype=np.int64)
    for d in range(D):
        half = T[d] // 2
        v = xl[d].astype(np.float64)
        dd = np.where(v < -half, -1, np.where(v >= half, 1, 0))
        delta[d] = dd
        code += (dd + 1) * 3 ** d
    return code, delta


def migrate(tile_of, xl, T, D, n):
    """Apply the migration rule to particles listed in (tile, old order).

    tile_of: (np,) tile id of each particle (array already grouped by tile in
    old order); xl: (D, np) unrebased local positions.  Returns
    (perm, new_tile, new_xl, counts): perm[k] = old index of the particle that
    lands at new position k, tiles in increasing id order."""
    nt = tile_grid(n, T, D)
    ntiles = nt[0] * nt[1] * nt[2]
    code, delta = direction(xl, T, D)
    centre_code = sum(3 ** d for d in range(D))
    tc = np.stack([tile_of % nt[0], (tile_of // nt[0]) % nt[1], tile_of // (nt[0] * nt[1])])
    dest_c = np.stack([(tc[d] + delta[d]) % nt[d] for d in range(3)])
    dest = tile_linear(dest_c, nt)
    # class 0 for stayers, 1 + code for arrivals, so that a stable sort by
    # (dest, class) over the old order yields the rule above
    cls = np.where(code == centre_code, 0, 1 + code)
    key = dest * (3 ** D + 2) + cls
    perm = np.argsort(key, kind="stable")
    new_xl = xl.copy()
    for d in range(D):
        new_xl[d] = (xl[d].astype(np.float64) - delta[d] * T[d]).astype(xl.dtype)
    counts = np.bincount(dest, minlength=ntiles)
    return perm, dest[perm], new_xl[:, perm], counts


def migration_counts(tile_before, tile_after, n, T, D, ntiles):
    """Per (tile before, direction code): how many particles moved from the
    tile to the neighbour at that offset (periodic tile grid), by direct
    counting over matched particles.  tile_before, tile_after: (np,) tile ids
    of the same particles before and after the step.  Needs at least 3 tiles
    along every grid dimension (with 2 the offsets -1 and +1 name the same
    tile)."""
    nt = tile_grid(n, T, D)
    assert all(nt[d] >= 3 for d in range(D)), "direction codes need >= 3 tiles per dimension"
    a = np.asarray(tile_before, dtype=np.int64)
    b = np.asarray(tile_after, dtype=np.int64)
    ca = [a % nt[0], (a // nt[0]) % nt[1], a // (nt[0] * nt[1])]
    cb = [b % nt[0], (b // nt[0]) % nt[1], b // (nt[0] * nt[1])]
    code = np.zeros(a.size, dtype=np.int64)
    for d in range(D):
        delta = (cb[d] - ca[d]) % nt[d]
        delta = np.where(delta == nt[d] - 1, -1, delta)   # one step at most
        if nt[d] == 1:
            delta = np.zeros_like(delta)
        code += (delta + 1) * 3 ** d
    out = np.zeros((ntiles, 3 ** D), dtype=np.int64)
    np.add.at(out, (a, code), 1)
    return out


def cell_sort(tile_of, xl, T, D):
    """Stable sort by (tile, cell key); returns the permutation."""
    key = tile_of.astype(np.int64) * int(np.prod([T[d] for d in range(D)])) + cell_key(xl, T, D)
    return np.argsort(key, kind="stable")


def to_global(tile_of, xl, n, T, D):
    """Global FP64 positions of tile-local coordinates (for comparisons)."""
    nt = tile_grid(n, T, D)
    tc = [tile_of % nt[0], (tile_of // nt[0]) % nt[1], tile_of // (nt[0] * nt[1])]
    out = np.zeros((D, xl.shape[1]))
    for d in range(D):
        out[d] = tc[d] * T[d] + T[d] // 2 + xl[d].astype(np.float64)
    return out
