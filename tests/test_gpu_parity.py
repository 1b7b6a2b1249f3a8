"""GPU-vs-oracle parity of every kernel of the step, through the C ABI.

Each test starts the HIP path and the FP64 oracle from one common state: the
GPU's own binned state (tile-local positions widened exactly to FP64 global
coordinates where the precision allows, fields widened from the working
precision).  Floating-point outputs must agree to relative L2 1e-12 (FP64
path) or 1e-5 (FP32 path); integer work (tile binning, migration order and
counts, cell sort) must be bit-exact.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import tiles

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5}


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def make_sim(plasma, T, prec, **kw):
    from paper_1906_06306_amd.sim import PicSim
    print(f"[gpu] PicSim D={plasma.D} n={plasma.n} T={T} prec={prec} np={plasma.nparticles}", flush=True)
    return PicSim(plasma, tile=T, precision=prec, **kw)


def common_state(sim, plasma):
    """Oracle state equal to what the GPU holds (widened to FP64)."""
    st = oracle.State(plasma)
    E, B, J = sim.fields_host(0)
    st.E[:] = E
    st.B[:] = B
    for s in range(len(plasma.species)):
        tid, xl, u = sim.particles_host(0, s)
        st.x[s] = np.ascontiguousarray(tiles.to_global(tid, xl, plasma.n, sim.T, plasma.D))
        st.u[s] = np.ascontiguousarray(u.astype(np.float64))
    return st


CASES = [
    # (D, n, T, ppc)
    (1, (96, 1, 1), (16, 1, 1), 24),
    (2, (48, 40, 1), (8, 8, 1), 6),
    (3, (16, 16, 12), (8, 8, 4), 2),
]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("D,n,T,ppc", CASES + [(2, (512, 320, 1), (2, 2, 1), 2)])
def test_init_binning_bit_exact(D, n, T, ppc, prec):
    """Binning against the oracle's rule, bit for bit; the last case has
    40,960 tiles in its box, beyond the 32,768 whose per-chunk histograms
    fit in LDS, so the binning kernels keep them in global memory."""
    plasma = synth.small_random(D, n, ppc, seed=3 + D)
    sim = make_sim(plasma, T, prec)
    dt = np.float64 if prec == "fp64" else np.float32
    counts = sim.counts_host()
    boxes = sim.state_boxes()
    ntiles = int(np.prod(tiles.tile_grid(n, T, D)))
    for s, sp in enumerate(plasma.species):
        tid, xl, order = tiles.bin_global(sp.x, n, T, D, dt)
        g_tid, g_xl, g_u = sim.particles_host(0, s)
        assert np.array_equal(g_tid, tid[order])
        assert np.array_equal(g_xl, xl[:, order])
        assert np.array_equal(g_u, sp.u[:, order].astype(dt))
        # per-tile counts, and the FP64 state read back: binning it again
        # gives the same tiles and local coordinates (an exact round trip)
        assert np.array_equal(counts[:ntiles, s], np.bincount(tid, minlength=ntiles))
        r_tid, r_xl, r_order = tiles.bin_global(boxes[0].pos[s], n, T, D, dt)
        assert np.array_equal(r_order, np.arange(r_tid.size))
        assert np.array_equal(r_tid, g_tid) and np.array_equal(r_xl, g_xl)
    E, B, J = sim.fields_host(0)
    assert np.array_equal(E, plasma.E.astype(dt).astype(np.float64))
    assert not J.any()
    d = sim.diagnostics()
    flags = sum(int(tiles.near_face(sim.particles_host(0, s)[1], D, T).sum()) for s in range(2))
    assert d["near_face"] == flags
    sim.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("D,n,T,ppc", CASES)
def test_unfused_step_stage_by_stage(D, n, T, ppc, prec):
    """Table-1 order through the separate entry points; each stage is
    compared with the oracle routine applied to the same inputs."""
    from paper_1906_06306_amd import _lib as L
    plasma = synth.small_random(D, n, ppc, seed=11 + D, field_amp=0.05)
    sim = make_sim(plasma, T, prec)
    st = common_state(sim, plasma)
    tol = TOL[prec]
    c = plasma.c
    # push_half_b1
    sim.fdtd(L.PIC_HALF_B)
    oracle.advance_b(D, n, 0.5 * c, st.E, st.B)
    E, B, _ = sim.fields_host(0)
    assert rel(B, st.B) < tol
    # interp_em + push (unfused: positions stay in their tile, unrebased)
    sim.push(fused=False)
    x_old = [x.copy() for x in st.x]
    disp = []
    for s in range(2):
        Ep, Bp = oracle.interp(D, n, st.E, st.B, st.x[s])
        oracle.boris(c, st.s[s], Ep, Bp, st.u[s])
        disp.append(oracle.move(D, c, st.u[s], st.x[s]))
        tid, xl, u, xo = sim.particles_host(0, s, with_xold=True)
        gx = tiles.to_global(tid, xl, n, T, D)
        assert rel(u.astype(np.float64), st.u[s]) < tol
        assert np.abs(gx - st.x[s]).max() < (1e-12 if prec == "fp64" else 4e-6 * max(T))
        assert np.array_equal(tiles.to_global(tid, xo, n, T, D), x_old[s])
    # push_half_b2
    sim.fdtd(L.PIC_HALF_B)
    oracle.advance_b(D, n, 0.5 * c, st.E, st.B)
    # comp_curr + halo fold
    sim.deposit()
    J = np.zeros_like(st.E)
    for s in range(2):
        oracle.zigzag(D, n, st.q[s], x_old[s], st.x[s], disp[s], J)
    _, B, Jg = sim.fields_host(0)
    assert rel(B, st.B) < tol
    assert rel(Jg, J) < tol, rel(Jg, J)
    # push_e + add_cur
    sim.fdtd(L.PIC_CURL_E_ADD_J)
    oracle.advance_e(D, n, c, st.B, st.E)
    oracle.add_current(n, J, st.E)
    E, _, _ = sim.fields_host(0)
    assert rel(E, st.E) < tol
    # particle communication: bit-exact against the rule applied to the
    # GPU's own pushed positions; migration counts by direct counting over
    # the particles matched through the rule's permutation
    before = [sim.particles_host(0, s) for s in range(2)]
    mc = sim.sort_migrate(counts=True)
    nt = tiles.tile_grid(n, T, D)
    for s in range(2):
        tid, xl, u = before[s]
        perm, ntid, nxl, counts = tiles.migrate(tid, xl, T, D, n)
        g_tid, g_xl, g_u = sim.particles_host(0, s)
        assert np.array_equal(g_tid, ntid)
        assert np.array_equal(g_xl, nxl)
        assert np.array_equal(g_u, u[:, perm])
        assert np.array_equal(np.bincount(g_tid, minlength=counts.size), counts)
        if min(nt[:D]) >= 3:
            want = tiles.migration_counts(tid[perm], ntid, n, T, D, counts.size)
            assert np.array_equal(mc[:, s, :], want)
        assert mc[:, s, :].sum() == tid.size
    assert sim.error() == 0
    sim.close()


@pytest.mark.parametrize("half_b_in_push", [False, True])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("D,n,T,ppc", CASES)
def test_fused_step_matches_oracle_and_unfused(D, n, T, ppc, prec, half_b_in_push):
    """One fused step (push + deposit + pack in one kernel, optionally with
    push_half_b1 done inside the push) against the oracle's full step, and
    its particle arrays against the unfused path."""
    plasma = synth.small_random(D, n, ppc, seed=21 + D, field_amp=0.05)
    sim = make_sim(plasma, T, prec)
    ref = make_sim(plasma, T, prec)
    st = common_state(sim, plasma)
    sim.step(1, fused=True, half_b_in_push=half_b_in_push)
    ref.step(1, fused=False)
    st.step(1)
    tol = TOL[prec]
    E, B, J = sim.fields_host(0)
    assert rel(B, st.B) < tol and rel(J, st.J) < tol and rel(E, st.E) < tol
    # same arithmetic in two kernels: identical tiles and order, values to
    # rounding (the compiler may contract multiply-adds differently)
    ptol = 1e-13 if prec == "fp64" else 1e-6
    for s in range(2):
        a = sim.particles_host(0, s)
        b = ref.particles_host(0, s)
        assert np.array_equal(a[0], b[0])
        assert np.abs(a[1] - b[1]).max() <= ptol * max(T)
        assert rel(a[2].astype(np.float64), b[2].astype(np.float64)) < ptol
    assert sim.error() == 0
    sim.close()
    ref.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("walls", [False, True])
@pytest.mark.parametrize("D,n,T,ppc", CASES)
def test_step_with_fold_and_e_in_one_pass_matches_separate_calls(D, n, T, ppc, prec, walls):
    """pic_step after a fused push folds the current blocks and applies
    E += c curl- B - J in one pass; the separate calls (fold, then the E
    update) compute the same values: bit for bit in FP32, whose current sums
    are exact, and to rounding in FP64 (LDS atomics add in no fixed order).
    Four steps, with and without conducting walls."""
    from paper_1906_06306_amd import _lib as L
    plasma = synth.small_random(D, n, ppc, theta=2.0 if walls else 0.3, seed=71 + D,
                                field_amp=0.05, q=0.01)
    a = make_sim(plasma, T, prec, walls=walls, capacity_factor=3.0)
    b = make_sim(plasma, T, prec, walls=walls, capacity_factor=3.0)
    for _ in range(4):
        a.step(1, fused=True, half_b_in_push=True)
        b.push(fused=True, half_b=True)
        b.fdtd(L.PIC_TWO_HALF_B)
        b.deposit()
        b.fdtd(L.PIC_CURL_E_ADD_J)
        b.sort_migrate()
    assert a.error() == 0 and b.error() == 0
    for x, y in zip(a.fields_host(0), b.fields_host(0)):
        if prec == "fp32":
            assert np.array_equal(x, y)
        else:
            assert rel(x, y) < 1e-13
    for s in range(2):
        pa, pb = a.particles_host(0, s), b.particles_host(0, s)
        assert np.array_equal(pa[0], pb[0])
        if prec == "fp32":
            assert np.array_equal(pa[1], pb[1]) and np.array_equal(pa[2], pb[2])
        else:
            assert np.abs(pa[1] - pb[1]).max() < 1e-12 and np.abs(pa[2] - pb[2]).max() < 1e-12
    a.close()
    b.close()


def test_fold_with_e_update_is_refused_under_fdtd4():
    """PIC_DEPOSIT_CURL_E carries the second-order E update: with FDTD4 the
    call fails with PIC_E_ARG and leaves the step where it was."""
    from paper_1906_06306_amd import _lib as L
    plasma = synth.small_random(2, (32, 32), 2, seed=5)
    sim = make_sim(plasma, (8, 8), "fp64", fdtd_order=4)
    sim.fdtd(L.PIC_HALF_B)
    sim.push(fused=True)
    sim.fdtd(L.PIC_HALF_B)
    with pytest.raises(L.PicError) as e:
        L.check(L.lib().pic_deposit_current(sim.ctx, L.PIC_ALL_SPECIES, L.PIC_DEPOSIT_CURL_E))
    assert e.value.code == L.PIC_E_ARG
    sim.deposit()
    sim.fdtd(L.PIC_CURL_E_ADD_J)
    sim.sort_migrate()
    assert sim.error() == 0
    sim.close()


def test_fp32_runs_are_bit_reproducible():
    """The FP32 push adds the current in 64-bit fixed point (exact integer
    adds), so the state after several steps does not depend on the order in
    which the LDS atomics, work-groups or walker iterations ran: the per-tile
    launch and the persistent walker give bit-identical fields and particles,
    and so do two runs of the same launch."""
    from paper_1906_06306_amd import _lib as L
    from paper_1906_06306_amd.sim import PicSim
    boxes = [synth.thermal_box(32, 48, 8, 0.3, seed=13), synth.thermal_box(64, 32, 16, 0.1, seed=14)]
    runs = [PicSim(boxes, tile=(16, 16), precision="fp32", options=o)
            for o in (0, 0, L.PIC_OPT_PERSISTENT)]
    for r in runs:
        r.step(5, half_b_in_push=True)
    for i in range(2):
        ref = runs[0].fields_host(i)
        for r in runs[1:]:
            for x, y in zip(ref, r.fields_host(i)):
                assert np.array_equal(x, y)
        for s in range(2):
            pa = runs[0].particles_host(i, s)
            for r in runs[1:]:
                pb = r.particles_host(i, s)
                assert all(np.array_equal(u, v) for u, v in zip(pa, pb))
    for r in runs:
        assert r.error() == 0
        r.close()


def test_regrow_continues_the_run_bit_for_bit():
    """A re-layout with larger segments (PicSim.regrow) holds the same state
    and, the FP32 current being exact, continues the run bit for bit."""
    plasma = synth.small_random(2, (64, 48), 4, seed=91, field_amp=0.05)
    sim = make_sim(plasma, (8, 8), "fp32", capacity_factor=1.5)
    sim.step(3, half_b_in_push=True)
    fill = sim.fill_ratio()
    big = sim.regrow(4.0)
    assert 0 < big.fill_ratio() < fill
    for x, y in zip(sim.fields_host(0)[:2], big.fields_host(0)[:2]):
        assert np.array_equal(x, y)
    for s in range(2):
        assert all(np.array_equal(a, b) for a, b in zip(sim.particles_host(0, s), big.particles_host(0, s)))
    sim.step(2, half_b_in_push=True)
    big.step(2, half_b_in_push=True)
    for x, y in zip(sim.fields_host(0), big.fields_host(0)):
        assert np.array_equal(x, y)
    for s in range(2):
        assert all(np.array_equal(a, b) for a, b in zip(sim.particles_host(0, s), big.particles_host(0, s)))
    assert sim.error() == 0 and big.error() == 0
    sim.close()
    big.close()


@pytest.mark.parametrize("block", [128, 256, 512])
@pytest.mark.parametrize("persistent", [False, True])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_uneven_segments_match_oracle(prec, persistent, block):
    """Segments of very different counts (the push visits them largest first,
    one work-group per (tile, species) segment, each with its own current
    block), at the work-group sizes the autotuner tries: three fused steps
    against the oracle, particle counts exact."""
    from paper_1906_06306_amd import _lib as L
    plasma = synth.small_random(2, (64, 48), 4, seed=77, field_amp=0.05)
    rng = np.random.default_rng(78)
    # 70% of the electrons into the 8x8 cells of one tile, 30% of the
    # positrons into another; the rest stay uniform
    for s, (frac, corner) in enumerate([(0.7, (16.0, 8.0)), (0.3, (40.0, 32.0))]):
        x = plasma.species[s].x
        k = rng.random(x.shape[1]) < frac
        x[0, k] = corner[0] + rng.random(int(k.sum())) * 8.0
        x[1, k] = corner[1] + rng.random(int(k.sum())) * 8.0
    T = (8, 8, 1)
    sim = make_sim(plasma, T, prec, tile_capacity="auto", capacity_factor=1.5, block=block,
                   options=L.PIC_OPT_PERSISTENT if persistent else 0)
    _, _, _, off, cnt = sim.particle_views()
    c = cnt.cpu().numpy()
    assert c.max() > 20 * np.median(c)          # the uneven case is really uneven
    tol = TOL[prec]
    for step in range(3):
        st = common_state(sim, plasma)          # each step from the GPU's own state
        sim.step(1, fused=True, half_b_in_push=True)
        st.step(1)
        E, B, J = sim.fields_host(0)
        assert rel(J, st.J) < tol and rel(E, st.E) < tol and rel(B, st.B) < tol, step
    assert sim.error() == 0
    _, _, _, off, cnt = sim.particle_views()
    c = cnt.cpu().numpy()
    assert [int(c[:, s].sum()) for s in range(2)] == [sp.x.shape[1] for sp in plasma.species]
    sim.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_cell_sort_bit_exact(prec):
    D, n, T = 2, (64, 32, 1), (16, 8, 1)
    plasma = synth.small_random(D, n, 5, seed=5)
    sim = make_sim(plasma, T, prec)
    sim.step(1, fused=True)
    before = [sim.particles_host(0, s) for s in range(2)]
    sim.sort_migrate(sort_cells=True)
    nf = 0
    for s in range(2):
        tid, xl, u = before[s]
        perm = tiles.cell_sort(tid, xl, T, D)
        g = sim.particles_host(0, s)
        assert np.array_equal(g[0], tid[perm]) and np.array_equal(g[1], xl[:, perm])
        assert np.array_equal(g[2], u[:, perm])
        nf += int(tiles.near_face(g[1], D, T).sum())
    assert sim.diagnostics()["near_face"] == nf
    sim.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_multistep_invariants(prec):
    """Gauss's law and div B through 20 fused steps (diagnostics in FP64);
    the FP32 path keeps them at FP32 round-off of the stored fields."""
    plasma = synth.turbulence(n=64, ppc=4, seed=9)
    sim = make_sim(plasma, (16, 16), prec)
    d0 = sim.diagnostics()
    sim.step(20, fused=True)
    d = sim.diagnostics()
    tol = 1e-12 if prec == "fp64" else 2e-5
    assert d["status"] == 0
    assert d["gauss_max"] < tol and d["divb_max"] < tol * max(1.0, 10 * abs(plasma.meta["B0"]))
    assert d["particles"] == d0["particles"] == plasma.nparticles
    assert abs(d["charge_total"]) < 1e-9
    sim.close()


def test_multibox_matches_single_boxes():
    """Two boxes of different sizes in one batch step exactly like each box
    alone (FP64)."""
    from paper_1906_06306_amd.sim import PicSim
    a = synth.thermal_box(32, 48, 3, 0.2, seed=1)
    b = synth.thermal_box(64, 16, 2, 0.05, seed=2)
    for p in (a, b):
        p.E[:] = 0.01 * np.random.default_rng(0).standard_normal(p.E.shape)
    batch = PicSim([a, b], tile=(16, 16), precision="fp64")
    one = [PicSim(p, tile=(16, 16), precision="fp64") for p in (a, b)]
    batch.step(3)
    for i, s1 in enumerate(one):
        s1.step(3)
        for x, y in zip(batch.fields_host(i), s1.fields_host(0)):
            assert rel(x, y) < 1e-13
        # LDS atomics add in no fixed order, so values agree to rounding
        for s in range(2):
            a, b_ = batch.particles_host(i, s), s1.particles_host(0, s)
            assert np.array_equal(a[0], b_[0])
            assert np.abs(a[1] - b_[1]).max() < 1e-12 and np.abs(a[2] - b_[2]).max() < 1e-12
        s1.close()
    batch.close()


def test_capacity_overflow_is_reported():
    """A segment too small for its particles latches PIC_E_CAPACITY at init
    (forced from the host with a tiny capacity; no kernel goes out of
    bounds)."""
    from paper_1906_06306_amd import _lib as L
    # 16 particles per cell per species: 1024 per 8x8 tile, against segments
    # of 256 (the requested 64 rounded up to the push kernel's group)
    plasma = synth.small_random(2, (32, 32), 16, seed=1)
    nt = 4 * 4
    cap = np.full((nt, 2), 64, dtype=np.int64)
    with pytest.raises(L.PicError) as e:
        make_sim(plasma, (8, 8), "fp32", tile_capacity=cap)
    assert e.value.code & L.PIC_E_CAPACITY


def test_outbox_overflow_is_reported():
    """More leavers in a step than a segment's outbox holds latch
    PIC_E_CAPACITY (forced from the host with the smallest outbox, 64 slots,
    against ~100 leavers per 8x8 tile of a hot plasma at 32 particles per
    cell; the push checks every outbox slot)."""
    from paper_1906_06306_amd import _lib as L
    plasma = synth.small_random(2, (32, 32), 32, theta=1.0, seed=5)
    sim = make_sim(plasma, (8, 8), "fp32", outbox_capacity=1, capacity_factor=2.0)
    assert sim.layout.outbox_capacity == 64
    sim.step(1, fused=True, half_b_in_push=True)
    assert sim.error() & L.PIC_E_CAPACITY
    sim.close()


def test_arrivals_beyond_capacity_are_reported():
    """A segment that receives more particles than its free slots latches
    PIC_E_CAPACITY in the migration (forced from the host: every segment
    holds exactly its capacity, the left half of the box streams into the
    right half at rest; the migration checks every destination slot)."""
    from paper_1906_06306_amd import _lib as L
    plasma = synth.small_random(2, (32, 32), 16, field_amp=0.0, seed=6)
    for sp in plasma.species:
        sp.u[:] = 0.0
        sp.u[0, sp.x[0] < 16.0] = 3.0
    cap = np.full((16, 2), 1024, dtype=np.int64)          # 16 per cell x 64 cells, a multiple of 64
    sim = make_sim(plasma, (8, 8), "fp32", tile_capacity=cap, block=64)
    assert sim.error() == 0
    sim.step(1, fused=True, half_b_in_push=True)
    assert sim.error() & L.PIC_E_CAPACITY
    sim.close()


def test_positions_outside_box_are_reported():
    from paper_1906_06306_amd import _lib as L
    plasma = synth.small_random(2, (32, 32), 2, seed=2)
    plasma.species[0].x[0, 5] = 40.0
    with pytest.raises(L.PicError) as e:
        make_sim(plasma, (8, 8), "fp32")
    assert e.value.code & L.PIC_E_OUT_OF_TILE


def test_persistent_walker_matches_per_tile_push():
    """The persistent tile walker (atomic work counter over the heaviest-first
    tile order) computes what the one-work-group-per-tile launch computes,
    on a batch of boxes with uneven tile loads (FP64)."""
    from paper_1906_06306_amd import _lib as L
    from paper_1906_06306_amd.sim import PicSim
    boxes = [synth.thermal_box(32, 48, 2, 0.2, seed=3), synth.thermal_box(64, 32, 6, 0.05, seed=4),
             synth.thermal_box(16, 16, 12, 1.0, seed=5)]
    a = PicSim(boxes, tile=(16, 16), precision="fp64")
    b = PicSim(boxes, tile=(16, 16), precision="fp64", options=L.PIC_OPT_PERSISTENT)
    a.step(4, half_b_in_push=True)
    b.step(4, half_b_in_push=True)
    for i in range(3):
        for x, y in zip(a.fields_host(i), b.fields_host(i)):
            assert rel(y, x) < 1e-13
        for s in range(2):
            pa, pb = a.particles_host(i, s), b.particles_host(i, s)
            assert np.array_equal(pa[0], pb[0])
            assert np.abs(pa[1] - pb[1]).max() < 1e-12 and np.abs(pa[2] - pb[2]).max() < 1e-12
    assert a.error() == 0 and b.error() == 0
    a.close()
    b.close()


@pytest.mark.parametrize("persistent", [False, True])
def test_graph_replays_match_eager_steps(persistent):
    """Three fused steps captured in a HIP graph, replayed three times with
    eager diagnostics (synchronising) between replays; every replay agrees
    with the same steps run eagerly (FP64, to rounding of LDS atomics)."""
    from paper_1906_06306_amd import _lib as L
    from paper_1906_06306_amd.sim import PicSim
    plasma = synth.turbulence(n=64, ppc=4, seed=12)
    opt = L.PIC_OPT_PERSISTENT if persistent else 0
    s1 = torch.cuda.Stream()
    s2 = torch.cuda.Stream()
    g = PicSim(plasma, tile=(16, 16), precision="fp64", options=opt, stream=s1)
    e = PicSim(plasma, tile=(16, 16), precision="fp64", options=opt, stream=s2)
    g.capture(3)            # one eager step, then 3 captured
    e.step(1, half_b_in_push=True)
    for rep in range(3):
        g.replay(1)
        e.step(3, half_b_in_push=True)
        dg, de = g.diagnostics(), e.diagnostics()
        assert dg["status"] == 0 and de["status"] == 0
        assert dg["particles"] == de["particles"] == plasma.nparticles
        for x, y in zip(g.fields_host(0), e.fields_host(0)):
            assert rel(x, y) < 1e-12, rep
        assert dg["gauss_max"] < 1e-12
    g.close()
    e.close()
