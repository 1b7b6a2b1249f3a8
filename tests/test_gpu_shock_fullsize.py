"""Parity of the 3D3V shock at its full size (1024 x 128 x 128 cells,
469.8 M particles), in the launch configuration its benchmark times: FP32,
8^3 tiles, the per-tile push with 512-thread work-groups, conducting walls
in x, segment capacities twice the dilated initial counts; every step is
the fused sequence (push with push_half_b1 in LDS, the two half B updates,
fold with the E update, migration).  Both push launches the benchmark
times are checked: one work-group per segment, and the persistent walker.

After 3 steps from the generated state (E and B no longer zero) one more
step is checked against the oracle on sampled tiles, from the GPU's own
state before it:

* B on every cell (it does not depend on the particles of the step);
* u and x of every particle that starts in the 27 tiles around each
  sampled centre tile, matched across the migration through origin ids;
* J and E on every cell of the centre tiles: every particle that deposits
  there starts within two cells of the tile, so inside its 27 tiles.

The centre tiles sit at least two tiles from the walls (no particle of
their neighbourhoods reaches a wall in one step, so the periodic interp
and ZigZag of the oracle apply), in the dense downstream, on both sides of
the density jump at x = 256, in the upstream beam and on the periodic seams
in y and z.  Cell decisions taken differently in FP32 and FP64 (an end point
within rounding of a cell face) are handled as in the 2D full-size test:
the oracle deposits such a particle from the kernel's end point, and every
one of them must be flagged near a face.  Relative L2 1e-5.

A second test takes the first step from the FP64 input itself (the
FP32/FP64 cell rule at full size in 3D): cells may differ from the
oracle's FP64 step only at particles flagged near a face.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import tiles

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-5
N3 = (1024, 128, 128)
T3 = (8, 8, 8)
# centre tiles (tx, ty, tz) of the 128 x 16 x 16 tile grid
CENTRES = [(2, 0, 0), (31, 15, 7), (32, 8, 15), (64, 3, 12), (100, 15, 15), (125, 0, 9)]


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def tile_id(nt, tx, ty, tz):
    return tx + nt[0] * ((ty % nt[1]) + nt[1] * (tz % nt[2]))


def around(nt, centre, r):
    tx, ty, tz = centre
    assert r <= tx < nt[0] - r           # the x range stays inside the walls
    return {tile_id(nt, tx + a, ty + b, tz + c)
            for a in range(-r, r + 1) for b in range(-r, r + 1) for c in range(-r, r + 1)}


def cells_of(n, T, nt, t):
    """Linear cell indices (x fastest) of tile t."""
    tc = [t % nt[0], (t // nt[0]) % nt[1], t // (nt[0] * nt[1])]
    i = tc[0] * T[0] + np.arange(T[0])
    j = tc[1] * T[1] + np.arange(T[1])
    k = tc[2] * T[2] + np.arange(T[2])
    return (i[None, None, :] + n[0] * (j[None, :, None] + n[1] * k[:, None, None])).reshape(-1)


def slots_and_tiles(off, cnt, s, tile_set):
    ts = np.array(sorted(tile_set), dtype=np.int64)
    sl = [np.arange(off[t, s], off[t, s] + cnt[t, s]) for t in ts]
    tid = [np.full(int(cnt[t, s]), t, dtype=np.int64) for t in ts]
    sl, tid = np.concatenate(sl), np.concatenate(tid)
    o = np.argsort(sl, kind="stable")                # slots in increasing order
    return sl[o], tid[o]


@pytest.mark.parametrize("walker", ["per_tile", "persistent"])
def test_shock_full_size_sampled_tiles(walker):
    from paper_1906_06306_amd import _lib as L
    from paper_1906_06306_amd.sim import PicSim
    n, T, D = N3, T3, 3
    nt = tiles.tile_grid(n, T, D)
    plasma = synth.shock()
    c = plasma.c
    q = [sp.q for sp in plasma.species]
    sgn = [sp.s for sp in plasma.species]
    print(f"[gpu] shock {n}, {plasma.nparticles} particles, FP32, T=8^3, block 512, walls, {walker}", flush=True)
    opts = L.PIC_OPT_TRACK | (L.PIC_OPT_PERSISTENT if walker == "persistent" else 0)
    sim = PicSim(plasma, tile=T, precision="fp32", tile_capacity="auto", capacity_factor=2.0,
                 options=opts, walls=True, block=512)
    del plasma
    sim.step(3, fused=True, half_b_in_push=True)
    assert sim.error() == 0
    E0, B0, _ = sim.fields_host(0)
    assert np.abs(E0).max() > 0 and np.abs(B0).max() > 0
    pos, u, _, off, cnt = sim.particle_views()
    ids_dev = sim.ids_view()
    inner = set().union(*[around(nt, ct, 1) for ct in CENTRES])
    outer = set().union(*[around(nt, ct, 2) for ct in CENTRES])
    offh, cnth = off.cpu().numpy(), cnt.cpu().numpy()
    pre = []
    for s in range(2):
        sl, tid = slots_and_tiles(offh, cnth, s, inner)
        it = torch.as_tensor(sl, device=sim.device)
        x = tiles.to_global(tid, pos[:, it].cpu().numpy(), n, T, D)
        pre.append((sl, x, u[:, it].cpu().numpy().astype(np.float64)))

    sim.step(1, fused=True, half_b_in_push=True)
    assert sim.error() == 0
    total, flagged = sim.sort_migrate(flagged_capacity=1 << 22)     # a sort-only call: nothing moves
    assert total <= 1 << 22
    flagged = np.sort(flagged)
    E1, B1, J1 = sim.fields_host(0)
    offh, cnth = off.cpu().numpy(), cnt.cpu().numpy()

    # the oracle's step from the GPU's state: B on the whole lattice
    Bh = B0.copy()
    oracle.advance_b(D, n, 0.5 * c, E0, Bh)                  # push_half_b1
    Bf = Bh.copy()
    oracle.advance_b(D, n, 0.5 * c, E0, Bf)                  # push_half_b2
    Ef = E0.copy()
    oracle.advance_e(D, n, c, Bf, Ef)                        # push_e
    J = np.zeros_like(E0)
    realigned = unflagged = 0
    for s in range(2):
        sl0, x1, uo = pre[s]
        Ep, Bp = oracle.interp(D, n, E0, Bh, x1)
        oracle.boris(c, sgn[s], Ep, Bp, uo)
        x2 = np.ascontiguousarray(x1.copy())
        disp = oracle.move(D, c, uo, x2)
        # the same particles after the step: somewhere in the 5^3 tiles
        sl1, tid1 = slots_and_tiles(offh, cnth, s, outer)
        it = torch.as_tensor(sl1, device=sim.device)
        origin = ids_dev[it].cpu().numpy().astype(np.int64)
        j = np.searchsorted(sl0, origin)
        j = np.minimum(j, sl0.size - 1)
        mine = sl0[j] == origin
        k = j[mine]
        assert np.unique(k).size == k.size == sl0.size, (s, k.size, sl0.size)
        it = torch.as_tensor(sl1[mine], device=sim.device)
        xg = tiles.to_global(tid1[mine], pos[:, it].cpu().numpy(), n, T, D)
        u1 = u[:, it].cpu().numpy().astype(np.float64)
        xk = xg.copy()
        for d in (1, 2):                                     # unwrap across the periodic seams
            xk[d] += n[d] * np.round((x2[d, k] - xg[d]) / n[d])
        dx = np.abs(xk - x2[:, k]).max()
        assert dx < 4e-6, (s, dx)
        assert rel(u1, uo[:, k]) < TOL, (s, rel(u1, uo[:, k]))
        diff = (np.floor(xk) != np.floor(x2[:, k])).any(axis=0)
        realigned += int(diff.sum())
        unflagged += int((~np.isin(sl1[mine][diff], flagged)).sum())
        x2[:, k[diff]] = xk[:, diff]
        oracle.zigzag(D, n, q[s], x1, np.ascontiguousarray(x2), disp, J)
    oracle.add_current(n, J, Ef)                             # add_cur
    cw = np.arange(0, int(np.prod(n)), n[0])                 # the wall planes
    Ef[1, cw] = Ef[2, cw] = 0.0
    Bf[0, cw] = 0.0
    cells = np.concatenate([cells_of(n, T, nt, tile_id(nt, *ct)) for ct in CENTRES])
    rj, re, rb = rel(J1[:, cells], J[:, cells]), rel(E1[:, cells], Ef[:, cells]), rel(B1, Bf)
    print(f"[gpu] shock full size: {sum(p[0].size for p in pre)} particles checked, {realigned} end points "
          f"in another cell than the oracle's ({total} flagged); rel L2 J {rj:.2e} E {re:.2e} (centre "
          f"tiles), B {rb:.2e} (lattice)", flush=True)
    assert unflagged == 0
    assert np.abs(J[:, cells]).max() > 0
    assert rj < TOL and re < TOL and rb < TOL
    sim.close()
    del sim
    torch.cuda.empty_cache()


def test_shock_full_size_fp32_cells_vs_fp64_input():
    """The FP32/FP64 cell rule at full size in 3D: one FP32 step from the
    FP64 input (positions rounded to FP32 tile-local coordinates at init)
    against the oracle's FP64 step from the same input, for every particle
    that ends in the 27 tiles around the sampled centres (matched through
    origin ids to its input index).  Cells may differ only at particles
    flagged near a face after the FP32 step; an unflagged mismatch fails."""
    from paper_1906_06306_amd import _lib as L
    from paper_1906_06306_amd.sim import PicSim
    n, T, D = N3, T3, 3
    nt = tiles.tile_grid(n, T, D)
    plasma = synth.shock()
    c = plasma.c
    print(f"[gpu] shock {n} from the FP64 input, {plasma.nparticles} particles, FP32", flush=True)
    sim = PicSim(plasma, tile=T, precision="fp32", tile_capacity="auto", capacity_factor=2.0,
                 options=L.PIC_OPT_TRACK, walls=True, block=512)
    ids_dev = sim.ids_view()
    ids0 = ids_dev.clone()                 # after init: index in the concatenated input
    sim.step(1, fused=True, half_b_in_push=True)
    assert sim.error() == 0
    total, flagged = sim.sort_migrate(flagged_capacity=1 << 22)
    assert total <= 1 << 22
    flagged = np.sort(flagged)
    pos, u, _, off, cnt = sim.particle_views()
    offh, cnth = off.cpu().numpy(), cnt.cpu().numpy()
    inner = set().union(*[around(nt, ct, 1) for ct in CENTRES])
    # the oracle's first step from the input: push_half_b1, interp, push
    Bh = np.ascontiguousarray(plasma.B, dtype=np.float64).copy()
    E0 = np.ascontiguousarray(plasma.E, dtype=np.float64)
    oracle.advance_b(D, n, 0.5 * c, E0, Bh)
    base = checked = mismatched = unflagged = 0
    for s, sp in enumerate(plasma.species):
        sl, tid = slots_and_tiles(offh, cnth, s, inner)
        it = torch.as_tensor(sl, device=sim.device)
        k = ids0[ids_dev[it].long()].cpu().numpy().astype(np.int64) - base
        base += sp.x.shape[1]
        assert (k >= 0).all() and (k < sp.x.shape[1]).all() and np.unique(k).size == k.size
        x1 = np.ascontiguousarray(sp.x[:, k])
        uo = np.ascontiguousarray(sp.u[:, k])
        Ep, Bp = oracle.interp(D, n, E0, Bh, x1)
        oracle.boris(c, sp.s, Ep, Bp, uo)
        x2 = x1.copy()
        oracle.move(D, c, uo, x2)
        xg = tiles.to_global(tid, pos[:, it].cpu().numpy(), n, T, D)
        for d in (1, 2):                                     # unwrap across the periodic seams
            xg[d] += n[d] * np.round((x2[d] - xg[d]) / n[d])
        assert np.abs(xg - x2).max() < 4e-6
        assert rel(u[:, it].cpu().numpy().astype(np.float64), uo) < TOL
        bad = (np.floor(xg) != np.floor(x2)).any(axis=0)
        checked += k.size
        mismatched += int(bad.sum())
        unflagged += int((~np.isin(sl[bad], flagged)).sum())
    print(f"[gpu] shock full size from the FP64 input: {checked} particles, {mismatched} cell mismatches, "
          f"{total} flagged, {unflagged} unflagged", flush=True)
    assert checked > 1_000_000
    assert unflagged == 0
    sim.close()
    del sim
    torch.cuda.empty_cache()
