"""Integer reporting of the particle-communication rows (Table 1) and the
per-species calls, through the C ABI.

* Migration counts [tiles][species][3^D] written by pic_sort_migrate after a
  fused step, against direct counting over every particle matched through
  its origin id (tile before -> tile after), FP32 and FP64, 2D and 3D.
* Near-face flags after every push: the count in the diagnostics and the
  flagged-slot list of pic_sort_migrate against the rule applied to the
  GPU's own positions (bit-exact).
* An FP32 step from the FP64 input against the oracle's FP64 step from the
  same input: every particle's cell agrees, except only at flagged
  particles (an unflagged mismatch fails).
* species_mask: pushing the species in separate calls gives exactly the
  one-call step; depositing one species gives that species' current.
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


def slots_of(sim, s):
    """Slots of species s in storage order (tiles in id order) and the tile
    of each."""
    _, _, _, off, cnt = sim.particle_views()
    off, cnt = off.cpu().numpy(), cnt.cpu().numpy()
    sl = [np.arange(off[t, s], off[t, s] + cnt[t, s]) for t in range(off.shape[0])]
    tl = [np.full(cnt[t, s], t) for t in range(off.shape[0])]
    return np.concatenate(sl), np.concatenate(tl)


CASES = [
    # (D, n, T, ppc, field amplitude)
    (2, (48, 40, 1), (8, 8, 1), 6, 0.05),
    (3, (24, 24, 24), (8, 8, 8), 2, 0.05),
]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("D,n,T,ppc,amp", CASES)
def test_fused_migration_counts_direct(D, n, T, ppc, amp, prec):
    from paper_1906_06306_amd import _lib as L
    from paper_1906_06306_amd.sim import PicSim
    plasma = synth.small_random(D, n, ppc, seed=31 + D, field_amp=amp)
    print(f"[gpu] migration counts D={D} n={n} T={T} {prec}", flush=True)
    sim = PicSim(plasma, tile=T, precision=prec, capacity_factor=2.0, options=L.PIC_OPT_TRACK)
    ntiles = int(sim.layout.tiles_total)
    for step in range(3):
        before = [slots_of(sim, s) for s in range(2)]
        tile_of_slot = np.full(int(sim.layout.capacity_total), -1, dtype=np.int64)
        for s in range(2):
            tile_of_slot[before[s][0]] = before[s][1]
        sim.push(fused=True, half_b=True)
        sim.fdtd(L.PIC_TWO_HALF_B)
        sim.deposit(curl_e=True)
        mc = sim.sort_migrate(counts=True)
        ids = sim.ids_host()
        moved = 0
        for s in range(2):
            sl, tl = slots_of(sim, s)
            origin = ids[sl]
            assert (origin >= 0).all()
            want = tiles.migration_counts(tile_of_slot[origin], tl, n, T, D, ntiles)
            assert np.array_equal(mc[:, s, :], want), (step, s)
            moved += int(want.sum() - want[:, sum(3 ** d for d in range(D))].sum())
        assert moved > 0
    assert sim.error() == 0
    sim.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("D,n,T,ppc,amp", CASES)
def test_near_face_flags_after_push(D, n, T, ppc, amp, prec):
    """The per-push count and the flagged list agree with the rule on the
    GPU's own stored positions, step after step; a position placed exactly
    on a face is always among them."""
    from paper_1906_06306_amd.sim import PicSim
    plasma = synth.small_random(D, n, ppc, seed=41 + D, field_amp=amp)
    # put some particles exactly on a face, and some 1e-9 off a face
    x = plasma.species[0].x
    x[:, :40] = np.floor(x[:, :40])
    x[0, 40:80] = np.floor(x[0, 40:80]) + 1e-9
    plasma.species[1].x[:] = x                       # co-located pairs stay neutral
    sim = PicSim(plasma, tile=T, precision=prec, capacity_factor=2.0)
    for step in range(4):
        if step:
            sim.step(1, fused=True, half_b_in_push=True)
        want, slots_want = 0, []
        for s in range(2):
            tid, xl, u = sim.particles_host(0, s)
            f = tiles.near_face(xl, D, T)
            want += int(f.sum())
            sl, _ = slots_of(sim, s)
            slots_want.append(sl[f])
        d = sim.diagnostics()
        assert d["near_face"] == want, (step, d["near_face"], want)
        if step == 0:
            assert want >= 40
        # the list (a sort-only call: nothing moves)
        total, lst = sim.sort_migrate(flagged_capacity=want + 5)
        assert total == want
        assert np.array_equal(np.sort(lst), lst)
        assert np.array_equal(lst, np.sort(np.concatenate(slots_want)))
        # a short list is cut, the total still exact
        total2, lst2 = sim.sort_migrate(flagged_capacity=max(want // 2, 1))
        assert total2 == want and np.array_equal(lst2, lst[:max(want // 2, 1)][:total2])
    assert sim.error() == 0
    sim.close()


def test_fp32_cells_match_fp64_oracle_except_flagged():
    """C-25 against oracle positions: an FP32 step from the FP64 input and
    the oracle's FP64 step from the same input put every particle in the
    same cell, except at particles flagged near a face after the FP32 step;
    an unflagged mismatch fails.  2D turbulence 256^2, 16 ppc/species
    (2.1 M particles), tile 16."""
    from paper_1906_06306_amd import _lib as L
    from paper_1906_06306_amd.sim import PicSim
    n, T = 256, (16, 16, 1)
    plasma = synth.turbulence(n=n, ppc=16, seed=17)
    print(f"[gpu] C-25 turbulence {n}^2 {plasma.nparticles} particles", flush=True)
    sim = PicSim(plasma, tile=T[:2], precision="fp32", capacity_factor=3.0, options=L.PIC_OPT_TRACK)
    ids0 = sim.ids_host()            # after init: index in the concatenated input
    sim.step(1, fused=True, half_b_in_push=True)
    total, flagged = sim.sort_migrate(flagged_capacity=1 << 20)
    assert total <= 1 << 20
    flagged = set(flagged.tolist())
    st = oracle.State(plasma)
    st.step(1)
    ids = sim.ids_host()             # after the step: the slot before it
    dims = (n, n, 1)
    base = 0
    mismatched = unflagged = 0
    for s in range(2):
        tid, xl, u = sim.particles_host(0, s)
        sl, _ = slots_of(sim, s)
        xg = tiles.to_global(tid, xl, dims, T, 2)
        # the oracle's particle that each slot holds
        k = ids0[ids[sl]] - base
        base += plasma.species[s].x.shape[1]
        xo = st.x[s][:, k]
        cg = np.floor(xg).astype(np.int64)
        co = np.floor(xo).astype(np.int64)
        bad = (cg != co).any(axis=0)
        mismatched += int(bad.sum())
        unflagged += sum(1 for j in np.nonzero(bad)[0] if int(sl[j]) not in flagged)
    print(f"[gpu] C-25: {mismatched} cell mismatches, {total} flagged, {unflagged} unflagged mismatches",
          flush=True)
    assert unflagged == 0
    assert sim.error() == 0
    sim.close()


@pytest.mark.parametrize("fused", [True, False])
@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_species_in_separate_calls(prec, fused):
    """Table 1 runs interp_em, push and comp_curr per particle container:
    two pushes with one species each, then one deposit of both, give exactly
    the single-call step (fields and particles, bit for bit in FP32), with
    the fused push and with the separate deposit."""
    from paper_1906_06306_amd import _lib as L
    from paper_1906_06306_amd.sim import PicSim
    plasma = synth.turbulence(n=64, ppc=4, seed=23)
    a = PicSim(plasma, tile=(16, 16), precision=prec)
    b = PicSim(plasma, tile=(16, 16), precision=prec)
    for _ in range(3):
        if fused:
            a.step(1, fused=True, half_b_in_push=True)
            b.push(fused=True, half_b=True, species=[1])
            b.push(fused=True, half_b=True, species=[0])
            b.fdtd(L.PIC_TWO_HALF_B)
        else:
            a.step(1, fused=False)
            b.fdtd(L.PIC_HALF_B)
            b.push(fused=False, species=[1])
            b.push(fused=False, species=[0])
            b.fdtd(L.PIC_HALF_B)
        b.deposit(curl_e=True)
        b.sort_migrate()
    # FP32 current blocks add exact fixed-point integers; FP64 blocks add in
    # the (unordered) order of the LDS atomics, so FP64 agrees to rounding
    exact = prec == "fp32"
    for x, y in zip(a.fields_host(0), b.fields_host(0)):
        assert np.array_equal(x, y) if exact else rel(y, x) < 1e-13
    for s in range(2):
        pa, pb = a.particles_host(0, s), b.particles_host(0, s)
        assert np.array_equal(pa[0], pb[0])
        for x, y in zip(pa[1:], pb[1:]):
            assert np.array_equal(x, y) if exact else np.abs(x - y).max() < 1e-12
    if exact:
        assert a.diagnostics()["near_face"] == b.diagnostics()["near_face"]
    a.close()
    b.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_deposit_of_one_species(prec):
    """Depositing only the positrons gives the oracle's ZigZag current of the
    positrons alone (unfused and fused)."""
    from paper_1906_06306_amd import _lib as L
    from paper_1906_06306_amd.sim import PicSim
    D, n, T = 2, (48, 40, 1), (8, 8, 1)
    plasma = synth.small_random(D, n, 5, seed=29, field_amp=0.05)
    for fused in (False, True):
        sim = PicSim(plasma, tile=T, precision=prec)
        st = oracle.State(plasma)
        E, B, _ = sim.fields_host(0)
        st.E[:], st.B[:] = E, B
        for s in range(2):
            tid, xl, u = sim.particles_host(0, s)
            st.x[s] = np.ascontiguousarray(tiles.to_global(tid, xl, n, T, D))
            st.u[s] = np.ascontiguousarray(u.astype(np.float64))
        oracle.advance_b(D, n, 0.5 * plasma.c, st.E, st.B)
        sim.fdtd(L.PIC_HALF_B)
        sim.push(fused=fused)
        sim.deposit(species=[1])
        Ep, Bp = oracle.interp(D, n, st.E, st.B, st.x[1])
        oracle.boris(plasma.c, st.s[1], Ep, Bp, st.u[1])
        x2 = st.x[1].copy()
        disp = oracle.move(D, plasma.c, st.u[1], x2)
        J = np.zeros_like(st.E)
        oracle.zigzag(D, n, st.q[1], st.x[1], x2, disp, J)
        _, _, Jg = sim.fields_host(0)
        assert rel(Jg, J) < TOL[prec], (fused, rel(Jg, J))
        sim.sort_migrate()
        assert sim.error() == 0
        sim.close()


def test_species_mask_errors():
    from paper_1906_06306_amd import _lib as L
    from paper_1906_06306_amd.sim import PicSim
    plasma = synth.small_random(2, (32, 32), 2, seed=2)
    sim = PicSim(plasma, tile=(8, 8), precision="fp32")
    lib = L.lib()
    assert lib.pic_push_interp(sim.ctx, 0, L.PIC_FUSED) == L.PIC_E_ARG           # empty
    assert lib.pic_push_interp(sim.ctx, 4, L.PIC_FUSED) == L.PIC_E_ARG           # beyond 2 species
    assert lib.pic_deposit_current(sim.ctx, 1, 0) == L.PIC_E_STATE               # nothing pushed
    assert lib.pic_push_interp(sim.ctx, 1, L.PIC_FUSED) == L.PIC_OK
    assert lib.pic_push_interp(sim.ctx, 1, L.PIC_FUSED) == L.PIC_E_STATE         # species 0 twice
    assert lib.pic_push_interp(sim.ctx, 2, 0) == L.PIC_E_STATE                   # unfused after fused
    assert lib.pic_deposit_current(sim.ctx, 3, 0) == L.PIC_E_STATE               # species 1 not pushed
    assert lib.pic_deposit_current(sim.ctx, 1, 0) == L.PIC_OK
    assert lib.pic_deposit_current(sim.ctx, 1, 0) == L.PIC_E_STATE               # once per step
    assert lib.pic_push_interp(sim.ctx, 2, L.PIC_FUSED) == L.PIC_E_STATE         # after the deposit
    assert lib.pic_sort_migrate(sim.ctx, 0, None, None, -1) == L.PIC_E_ARG
    assert lib.pic_sort_migrate(sim.ctx, 0, None, None, 0) == L.PIC_OK
    mc = torch.zeros(1024, dtype=torch.int32, device="cuda")
    assert lib.pic_sort_migrate(sim.ctx, 0, mc.data_ptr(), None, 0) == L.PIC_E_STATE   # no push before
    assert sim.error() == 0
    sim.close()
