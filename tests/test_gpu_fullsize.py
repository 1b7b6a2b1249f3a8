"""Parity at the benchmark sizes, in the launch configuration bench.py
times (fused push with push_half_b1 in LDS, tile edge 16).

* Decaying turbulence, 1024^2 cells, 16 particles per cell per species
  (33.5 M particles), one step from the GPU's own state after 5 steps (E
  no longer zero), FP32 and FP64,
  against the oracle on the whole lattice: E, B and J on every cell, u and x
  of every particle (matched across the migration through origin ids).
  Where floating point decides an integer, both sides take the decision in
  the kernel's precision: the few particles whose end point the oracle puts
  in another cell than the kernel does (an end point within rounding of a
  cell face, where App. D's relay point jumps from the midpoint to the face)
  are deposited by the oracle from the kernel's end point; every one of them
  must be flagged near a face (an unflagged one fails).  Relative L2 1e-5
  (FP32) and 1e-12 (FP64).
* The same workload from the FP64 input: the FP32 step's cells match the
  oracle's FP64 step except at flagged particles.
* The 1D3V two-stream (Weibel-shaped) workload, 512 cells, 64 particles per
  cell per species, FP64, its full 200 steps: Gauss's law and div B hold to
  round-off on the GPU, and the fields stay close to the oracle's own run.
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
    _, _, _, off, cnt = sim.particle_views()
    off, cnt = off.cpu().numpy(), cnt.cpu().numpy()
    return np.concatenate([np.arange(off[t, s], off[t, s] + cnt[t, s]) for t in range(off.shape[0])])


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_turbulence_full_size_whole_lattice(prec):
    from paper_1906_06306_amd import _lib as L
    from paper_1906_06306_amd.sim import PicSim
    n, T = 1024, (16, 16, 1)
    dims = (n, n, 1)
    plasma = synth.turbulence(n=n, ppc=16)
    print(f"[gpu] turbulence {n}^2, {plasma.nparticles} particles, {prec}, T=16, whole lattice", flush=True)
    sim = PicSim(plasma, tile=T[:2], precision=prec, capacity_factor=3.0, options=L.PIC_OPT_TRACK)
    sim.step(5, fused=True, half_b_in_push=True)
    E0, B0, _ = sim.fields_host(0)
    assert np.abs(E0).max() > 0
    pre = []
    for s in range(2):
        tid, xl, u = sim.particles_host(0, s)
        pre.append((slots_of(sim, s), tiles.to_global(tid, xl, dims, T, 2), u.astype(np.float64)))
    sim.step(1, fused=True, half_b_in_push=True)
    assert sim.error() == 0
    total, flagged = sim.sort_migrate(flagged_capacity=1 << 22)     # a sort-only call: nothing moves
    assert total <= 1 << 22
    flagged = np.sort(flagged)
    E1, B1, J1 = sim.fields_host(0)
    ids = sim.ids_host()
    c = plasma.c
    tol = TOL[prec]
    # the oracle's step, Table-1 order, from the GPU's state before the step
    st = oracle.State(plasma)
    st.E[:], st.B[:] = E0, B0
    for s in range(2):
        st.x[s] = np.ascontiguousarray(pre[s][1])
        st.u[s] = np.ascontiguousarray(pre[s][2])
    ends = st.push_particles()
    realigned = unflagged = 0
    for s in range(2):
        sl0 = pre[s][0]
        u, x2 = st.u[s], ends[s]
        tid1, xl1, u1 = sim.particles_host(0, s)
        sl1 = slots_of(sim, s)
        inv = np.full(ids.size, -1, dtype=np.int64)
        inv[sl0] = np.arange(sl0.size)
        k = inv[ids[sl1]]                              # oracle index of every stored particle
        assert (k >= 0).all() and np.unique(k).size == k.size == sl0.size
        xg = tiles.to_global(tid1, xl1, dims, T, 2)    # in [0, n)
        # the kernel's end point, unwrapped next to the oracle's
        xk = xg + n * np.round((x2[:, k] - xg) / n)
        dx = np.abs(xk - x2[:, k]).max()
        assert dx < (1e-12 if prec == "fp64" else 4e-6), dx
        assert rel(u1.astype(np.float64), u[:, k]) < tol
        # cells decided differently: deposit from the kernel's end point
        diff = (np.floor(xk) != np.floor(x2[:, k])).any(axis=0)
        realigned += int(diff.sum())
        unflagged += int((~np.isin(sl1[diff], flagged)).sum())
        x2[:, k[diff]] = xk[:, diff]
    st.finish_step(ends)
    E, B, J = st.E, st.B, st.J
    print(f"[gpu] {prec}: {realigned} end points in another cell than the oracle's ({total} flagged); "
          f"rel L2 E {rel(E1, E):.2e} B {rel(B1, B):.2e} J {rel(J1, J):.2e}", flush=True)
    assert unflagged == 0
    assert rel(J1, J) < tol and rel(E1, E) < tol and rel(B1, B) < tol
    sim.close()


def test_turbulence_full_size_fp32_cells_vs_fp64_input():
    """C-25 at full size: the FP32 step from the FP64 input against the
    oracle's FP64 step from the same input; cells differ only at flagged
    particles."""
    from paper_1906_06306_amd import _lib as L
    from paper_1906_06306_amd.sim import PicSim
    n, T = 1024, (16, 16, 1)
    dims = (n, n, 1)
    plasma = synth.turbulence(n=n, ppc=16)
    print(f"[gpu] C-25 turbulence {n}^2 from the FP64 input", flush=True)
    sim = PicSim(plasma, tile=T[:2], precision="fp32", capacity_factor=3.0, options=L.PIC_OPT_TRACK)
    ids0 = sim.ids_host()
    sim.step(1, fused=True, half_b_in_push=True)
    total, flagged = sim.sort_migrate(flagged_capacity=1 << 22)
    flagged = np.sort(flagged)
    ids = sim.ids_host()
    st = oracle.State(plasma)
    st.step(1)
    base = mism = unflagged = 0
    for s in range(2):
        tid, xl, _ = sim.particles_host(0, s)
        sl = slots_of(sim, s)
        k = ids0[ids[sl]] - base
        base += plasma.species[s].x.shape[1]
        xg = tiles.to_global(tid, xl, dims, T, 2)
        bad = (np.floor(xg) != np.floor(st.x[s][:, k])).any(axis=0)
        mism += int(bad.sum())
        unflagged += int((~np.isin(sl[bad], flagged)).sum())
    print(f"[gpu] C-25 full size: {mism} cell mismatches, {total} flagged, {unflagged} unflagged", flush=True)
    assert unflagged == 0
    assert sim.error() == 0
    sim.close()


def test_two_stream_full_run_fp64():
    from paper_1906_06306_amd.sim import PicSim
    plasma = synth.weibel()
    print(f"[gpu] two-stream 1D, {plasma.nparticles} particles, FP64, 200 steps", flush=True)
    sim = PicSim(plasma, tile=(32,), precision="fp64", capacity_factor=2.0)
    st = oracle.State(plasma)
    sim.step(200, fused=True, half_b_in_push=True)
    st.step(200)
    d = sim.diagnostics()
    assert d["status"] == 0 and d["particles"] == plasma.nparticles
    assert d["gauss_max"] < 1e-12 and d["divb_max"] < 1e-12
    E, B, J = sim.fields_host(0)
    uf, uk = st.energies()
    print(f"[gpu] after 200 steps: rel L2 E {rel(E, st.E):.3e}, field energy GPU {d['field_energy']:.6e} "
          f"oracle {uf:.6e}", flush=True)
    assert uf > 1e-6                       # the beams have driven fields
    # exponential growth amplifies round-off differences; 200 steps keep
    # them well below the field itself
    assert rel(E, st.E) < 1e-6
    assert abs(d["field_energy"] - uf) < 1e-6 * uf
    sim.close()
