"""Parity at the benchmark sizes, in the launch configuration bench.py
times (fused push with push_half_b1 in LDS, autotuned tile edge 16).

* Decaying turbulence, 1024^2 cells, 16 particles per cell per species
  (33.5 M particles), FP32, one step from the GPU's own state:
  - 20,000 sampled particles (matched across the migration through their
    origin ids) against the oracle's interpolation, Boris push and position
    update computed one by one on the same FP64-widened fields;
  - the current of 6 sampled tiles against the oracle's ZigZag deposit of
    every particle that started in the 3x3 tiles around each (only those
    reach the tile's cells);
  - E and B against the oracle's field updates with that current.
  Relative L2 1e-5 throughout.
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


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def test_turbulence_full_size_sampled_parity():
    from paper_1906_06306_amd import _lib as L
    from paper_1906_06306_amd.sim import PicSim
    n, T = 1024, (16, 16)
    plasma = synth.turbulence(n=n, ppc=16)
    print(f"[gpu] turbulence {n}^2, {plasma.nparticles} particles, FP32, T=16", flush=True)
    sim = PicSim(plasma, tile=T, precision="fp32", capacity_factor=3.0, options=L.PIC_OPT_TRACK)
    E0, B0, _ = sim.fields_host(0)
    pre = []
    for s in range(2):
        tid, xl, u = sim.particles_host(0, s)
        _, _, _, off, cnt = sim.particle_views()
        off, cnt = off.cpu().numpy(), cnt.cpu().numpy()
        slots = np.concatenate([np.arange(off[t, s], off[t, s] + cnt[t, s]) for t in range(off.shape[0])])
        pre.append((tid, xl, u, slots))
    sim.step(1, fused=True, half_b_in_push=True)
    assert sim.error() == 0
    E1, B1, J1 = sim.fields_host(0)
    ids = sim.ids_host()
    c = plasma.c
    dims = (n, n, 1)
    # B^n as the push sees it
    Bn = B0.copy()
    oracle.advance_b(2, dims, 0.5 * c, E0, Bn)
    rng = np.random.default_rng(5)
    nt = n // T[0]
    sample_tiles = rng.choice(nt * nt, 6, replace=False)
    for s in range(2):
        tid, xl, u, slots = pre[s]
        x0 = tiles.to_global(tid, xl, dims, T + (1,), 2)
        # sampled particles, one by one
        k = rng.choice(x0.shape[1], 10000, replace=False)
        Ep, Bp = oracle.interp(2, dims, E0, Bn, x0[:, k])
        uo = u[:, k].astype(np.float64).copy()
        oracle.boris(c, plasma.species[s].s, Ep, Bp, uo)
        xo = x0[:, k].copy()
        oracle.move(2, c, uo, xo)
        oracle.wrap(2, dims, xo)
        tid1, xl1, u1 = sim.particles_host(0, s)
        _, _, _, off, cnt = sim.particle_views()
        off, cnt = off.cpu().numpy(), cnt.cpu().numpy()
        slots1 = np.concatenate([np.arange(off[t, s], off[t, s] + cnt[t, s]) for t in range(off.shape[0])])
        inv = np.full(ids.size, -1, dtype=np.int64)
        inv[ids[slots1]] = np.arange(slots1.size)
        j = inv[slots[k]]
        assert (j >= 0).all()
        xg = tiles.to_global(tid1[j], xl1[:, j], dims, T + (1,), 2)
        dx = np.abs(xg - xo)
        dx = np.minimum(dx, n - dx)                   # periodic distance
        assert dx.max() < 5e-5, dx.max()
        assert rel(u1[:, j].astype(np.float64), uo) < 1e-5
    # the current on each sampled tile's cells: the oracle deposits every
    # particle that started in the 3x3 tiles around it
    for t in sample_tiles:
        cx, cy = t % nt, t // nt
        Jt = np.zeros_like(E0)
        for s in range(2):
            tid, xl, u, slots = pre[s]
            x0 = tiles.to_global(tid, xl, dims, T + (1,), 2)
            tx, ty = tid % nt, tid // nt
            near = (np.minimum((tx - cx) % nt, (cx - tx) % nt) <= 1) & (np.minimum((ty - cy) % nt, (cy - ty) % nt) <= 1)
            sel = np.nonzero(near)[0]
            Ep, Bp = oracle.interp(2, dims, E0, Bn, x0[:, sel])
            us = u[:, sel].astype(np.float64).copy()
            oracle.boris(c, plasma.species[s].s, Ep, Bp, us)
            x2 = x0[:, sel].copy()
            disp = oracle.move(2, c, us, x2)
            oracle.zigzag(2, dims, plasma.species[s].q, x0[:, sel], x2, disp, Jt)
        cells = np.array([(cy * T[1] + j) * n + cx * T[0] + i for j in range(T[1]) for i in range(T[0])])
        assert rel(J1[:, cells], Jt[:, cells]) < 1e-5, (t, rel(J1[:, cells], Jt[:, cells]))
    # fields with the GPU's current
    Be = Bn.copy()
    oracle.advance_b(2, dims, 0.5 * c, E0, Be)
    Ee = E0.copy()
    oracle.advance_e(2, dims, c, Be, Ee)
    oracle.add_current(dims, J1, Ee)
    assert rel(B1, Be) < 1e-5 and rel(E1, Ee) < 1e-5, (rel(B1, Be), rel(E1, Ee))
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
