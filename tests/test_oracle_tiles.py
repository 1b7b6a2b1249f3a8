"""Pins of the tile-level integer rules in oracle.tiles (P-12): brute-force
loops that build the same orderings element by element, exactness of the
centre-relative rebasing, and direct counting."""
import numpy as np
import pytest

from oracle import tiles
import synth


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("D", [1, 2, 3])
def test_bin_global_exact_and_stable(D, dtype):
    rng = np.random.default_rng(D)
    n = (32, 24, 16)[:D] + (1,) * (3 - D)
    T = (8, 6, 4)[:D] + (1,) * (3 - D)
    x = synth.quiet_positions(rng, D, n, 3)
    x = x[:, rng.permutation(x.shape[1])]
    # plant values that round onto the upper tile face in FP32
    x[0, 0] = 8.0 - 1e-9
    x[0, 1] = 4.0 - 1e-12
    tid, xl, order = tiles.bin_global(x, n, T, D, dtype)
    nt = tiles.tile_grid(n, T, D)
    # every local coordinate inside [-T/2, T/2)
    for d in range(D):
        assert (xl[d] >= -T[d] // 2).all() and (xl[d] < T[d] // 2).all()
    # global position recovered: exactly in FP64 away from the first tile
    # along each axis (there x - centre can need more bits than x has, since
    # |x| < T/2), to rounding elsewhere
    back = tiles.to_global(tid, xl, n, T, D)
    L = np.array(n[:D], float)[:, None]
    diff = back - x
    diff = np.where(diff > L / 2, diff - L, np.where(diff < -L / 2, diff + L, diff))
    ntx, nty = n[0] // T[0], n[1] // T[1]
    tc = np.stack([tid % ntx, (tid // ntx) % nty, tid // (ntx * nty)])[:D]
    interior = (tc >= 1).all(0)
    if dtype == np.float64:
        assert np.abs(diff[:, interior]).max() == 0.0
        assert np.abs(diff).max() <= 2.0 ** -52 * max(T)
    else:
        assert np.abs(diff).max() <= 2.0 ** -21 * max(T)
    if dtype == np.float32:
        assert tid[0] % nt[0] == 1 and xl[0, 0] == -4.0     # rounded up to the face: next tile
    # stable grouping, brute force
    brute = []
    for t in range(nt[0] * nt[1] * nt[2]):
        brute.extend([i for i in range(x.shape[1]) if tid[i] == t])
    assert np.array_equal(order, np.array(brute))


def test_migrate_matches_brute_force_lists():
    rng = np.random.default_rng(8)
    D, n, T = 2, (24, 16, 1), (8, 4, 1)
    x = synth.quiet_positions(rng, D, n, 2)
    tid, xl, order = tiles.bin_global(x, n, T, D, np.float32)
    tid, xl = tid[order], xl[:, order]
    # push every particle by up to 0.9 cells
    xl2 = (xl.astype(np.float64) + rng.uniform(-0.9, 0.9, xl.shape)).astype(np.float32)
    perm, ntid, nxl, counts = tiles.migrate(tid, xl2, T, D, n)
    nt = tiles.tile_grid(n, T, D)
    ntl = nt[0] * nt[1]
    # brute force: destination per particle
    dest, delta = [], []
    for i in range(tid.size):
        tx, ty = tid[i] % nt[0], tid[i] // nt[0]
        dx = -1 if xl2[0, i] < -4 else (1 if xl2[0, i] >= 4 else 0)
        dy = -1 if xl2[1, i] < -2 else (1 if xl2[1, i] >= 2 else 0)
        dest.append(((tx + dx) % nt[0]) + nt[0] * ((ty + dy) % nt[1]))
        delta.append((dx, dy))
    want = []
    for r in range(ntl):
        want += [i for i in range(tid.size) if tid[i] == r and dest[i] == r and delta[i] == (0, 0)]
        for code in range(9):
            if code == 4:
                continue
            dd = (code % 3 - 1, code // 3 - 1)
            want += [i for i in range(tid.size) if dest[i] == r and delta[i] == dd]
    assert np.array_equal(perm, np.array(want))
    assert np.array_equal(counts, np.bincount(np.array(dest), minlength=ntl))
    # rebasing is exact: the global position is unchanged (mod the box)
    g_old = tiles.to_global(tid, xl2, n, T, D)[:, perm]
    g_new = tiles.to_global(ntid, nxl, n, T, D)
    diff = (g_new - g_old) % np.array(n[:D], float)[:, None]
    diff = np.where(diff > 1, diff - np.array(n[:D], float)[:, None], diff)
    assert np.abs(diff).max() == 0.0
    for d in range(D):
        assert (nxl[d] >= -T[d] // 2).all() and (nxl[d] < T[d] // 2).all()


def test_cell_sort_and_keys_brute_force():
    rng = np.random.default_rng(12)
    D, n, T = 3, (8, 8, 8), (4, 4, 4)
    x = synth.quiet_positions(rng, D, n, 2)
    x = x[:, rng.permutation(x.shape[1])]
    tid, xl, order = tiles.bin_global(x, n, T, D, np.float32)
    tid, xl = tid[order], xl[:, order]
    key = tiles.cell_key(xl, T, D)
    for i in range(0, tid.size, 37):
        cx, cy, cz = [int(np.floor(xl[d, i])) + 2 for d in range(3)]
        assert key[i] == cx + 4 * (cy + 4 * cz)
    perm = tiles.cell_sort(tid, xl, T, D)
    want = sorted(range(tid.size), key=lambda i: (tid[i], key[i]))   # Python sort is stable
    assert np.array_equal(perm, np.array(want))


def test_near_face_flags():
    """The band is 2 ulps of the storage precision at the tile half-width:
    for T = 16 in FP32, 2 * 2^-20 around every integer, whatever the size of
    the coordinate itself."""
    f32 = np.float32
    h = 2.0 ** -20
    vals = [0.0, 1.5, f32(2.0) - f32(2.0 ** -23), -3.0, 0.25, f32(5 + 1.5 * h), f32(5 + 2.5 * h),
            f32(-7.0 - 2 * h), f32(-8.0), f32(7.9999995), f32(0.5 * h), f32(3 * h)]
    xl = np.array([vals], dtype=np.float32)
    f = tiles.near_face(xl, 1, (16, 1, 1))
    want = [True, False, True, True, False, True, False, True, True, True, True, False]
    assert f.tolist() == want
    # brute force over FP32 neighbours of a few integers: flagged exactly
    # when at most 2^-19 away
    for k in (-8, -3, 0, 1, 7):
        v = np.float32(k)
        up, dn = [v], [v]
        for _ in range(40):
            up.append(np.nextafter(up[-1], np.float32(np.inf)))
            dn.append(np.nextafter(dn[-1], np.float32(-np.inf)))
        xs = np.array([up + dn], dtype=np.float32)
        fl = tiles.near_face(xs, 1, (16, 1, 1))
        for val, got in zip(xs[0], fl):
            assert got == (abs(float(val) - k) <= 2 * h), (k, float(val))
    # FP64: the band is 2 ulp(8) = 2^-48
    xd = np.array([[3.0 + 2.0 ** -49, 3.0 + 2.0 ** -47]])
    assert tiles.near_face(xd, 1, (16, 1, 1)).tolist() == [True, False]


def test_migration_counts_brute_force():
    """P-12: counts per (tile, direction) from matched tile ids against a
    plain loop over the particles, including moves across the periodic seam."""
    rng = np.random.default_rng(4)
    n, T, D = (48, 40, 1), (8, 8, 1), 2
    nt = [6, 5, 1]
    ntiles = 30
    a = rng.integers(0, ntiles, 5000)
    delta = rng.integers(-1, 2, (2, 5000))
    ax, ay = a % 6, a // 6
    b = (ax + delta[0]) % 6 + 6 * ((ay + delta[1]) % 5)
    got = tiles.migration_counts(a, b, n, T, D, ntiles)
    want = np.zeros((ntiles, 9), dtype=np.int64)
    for i in range(a.size):
        want[a[i], (delta[0, i] + 1) + 3 * (delta[1, i] + 1)] += 1
    assert np.array_equal(got, want)
    assert got.sum() == a.size
