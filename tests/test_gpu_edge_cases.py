"""Degenerate inputs of the fused step against the oracle (one step at a
time from the state the GPU holds, particles matched through their origin
ids):

* one species empty, the other a thermal population;
* single particles that cross a tile corner diagonally, one of them across
  the periodic seam in both dimensions at once;
* particles started exactly on cell faces and tile faces;
* particles at rest in zero fields, half of them on faces: the current is
  exactly zero, nothing moves, and every particle on a face stays flagged
  as near a face;
* a NaN four-velocity, and a move of a whole cell at a Courant number of 1:
  the device error is latched and reported, the particle stays, and the
  rest of the step is the oracle's step of the other particles.
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


def plasma_of(D, n, xs, us, field_amp, seed, c=0.45, q=1e-3):
    """Pair plasma from explicit positions and momenta per species (lists of
    (D, np) and (3, np) arrays) with random E and B of amplitude field_amp."""
    rng = np.random.default_rng(seed)
    dims = tuple(n) + (1,) * (3 - len(n))
    N = int(np.prod(dims))
    E = field_amp * rng.standard_normal((3, N))
    B = field_amp * rng.standard_normal((3, N))
    sp = [synth.Species(q=-q, s=-1.0, m=q, x=np.ascontiguousarray(xs[0], dtype=np.float64),
                        u=np.ascontiguousarray(us[0], dtype=np.float64)),
          synth.Species(q=+q, s=+1.0, m=q, x=np.ascontiguousarray(xs[1], dtype=np.float64),
                        u=np.ascontiguousarray(us[1], dtype=np.float64))]
    return synth.Plasma(D=D, n=dims, c=c, species=sp, E=E, B=B, meta=dict(workload="edge"))


def slots_in_order(sim, s):
    _, _, _, off, cnt = sim.particle_views()
    off, cnt = off.cpu().numpy(), cnt.cpu().numpy()
    parts = [np.arange(off[t, s], off[t, s] + cnt[t, s]) for t in range(off.shape[0])]
    return np.concatenate(parts) if parts else np.zeros(0, dtype=np.int64)


def common_state(sim, plasma):
    st = oracle.State(plasma)
    E, B, _ = sim.fields_host(0)
    st.E[:], st.B[:] = E, B
    for s in range(2):
        tid, xl, u = sim.particles_host(0, s)
        st.x[s] = np.ascontiguousarray(tiles.to_global(tid, xl, plasma.n, sim.T, plasma.D))
        st.u[s] = np.ascontiguousarray(u.astype(np.float64))
    return st


def step_and_compare(sim, plasma, prec, steps):
    """`steps` fused steps, each from the GPU's own state, against the oracle."""
    D, n, T = plasma.D, plasma.n, sim.T
    tol = TOL[prec]
    for k in range(steps):
        st = common_state(sim, plasma)
        pre = [slots_in_order(sim, s) for s in range(2)]
        sim.step(1, fused=True, half_b_in_push=True)
        st.step(1)
        assert sim.error() == 0
        E, B, J = sim.fields_host(0)
        assert rel(J, st.J) < tol and rel(E, st.E) < tol and rel(B, st.B) < tol, (k, rel(J, st.J))
        ids = sim.ids_host()
        for s in range(2):
            tid, xl, u = sim.particles_host(0, s)
            assert xl.shape[1] == st.x[s].shape[1]
            if xl.shape[1] == 0:
                continue
            gx = tiles.to_global(tid, xl, n, T, D)
            origin = ids[slots_in_order(sim, s)]
            j = np.searchsorted(pre[s], origin)
            assert np.array_equal(pre[s][j], origin)
            ptol = 1e-12 if prec == "fp64" else 4e-6 * max(T)
            d = np.abs(gx - st.x[s][:, j])
            d = np.minimum(d, np.array(n[:D])[:, None] - d)       # across the periodic seam
            assert d.max() < ptol, (k, s, d.max())
            assert rel(u.astype(np.float64), st.u[s][:, j]) < tol


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_one_species_empty(prec):
    from paper_1906_06306_amd import _lib as L
    from paper_1906_06306_amd.sim import PicSim
    full = synth.small_random(2, (32, 24), 4, seed=41, field_amp=0.05)
    p = plasma_of(2, (32, 24), [full.species[0].x[:, :0], full.species[1].x],
                  [full.species[0].u[:, :0], full.species[1].u], 0.05, seed=42)
    print(f"[gpu] one species empty, {p.nparticles} particles, {prec}", flush=True)
    sim = PicSim(p, tile=(8, 8), precision=prec, capacity_factor=3.0, options=L.PIC_OPT_TRACK)
    step_and_compare(sim, p, prec, 3)
    d = sim.diagnostics()
    assert d["status"] == 0 and d["particles"] == p.nparticles
    sim.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_single_particles_cross_tile_corners(prec):
    """One electron crosses the corner of tiles (0,0) and (1,1) at (8, 8);
    one positron crosses the corner at the periodic seam (32, 0)."""
    from paper_1906_06306_amd import _lib as L
    from paper_1906_06306_amd.sim import PicSim
    xe = np.array([[7.95], [7.95]])
    ue = np.array([[0.6], [0.6], [0.1]])
    xp = np.array([[31.95], [0.05]])
    up = np.array([[0.6], [-0.6], [-0.2]])
    p = plasma_of(2, (32, 32), [xe, xp], [ue, up], 0.01, seed=43)
    print(f"[gpu] tile-corner crossings, {prec}", flush=True)
    sim = PicSim(p, tile=(8, 8), precision=prec, capacity_factor=2.0, options=L.PIC_OPT_TRACK)
    tid0 = [sim.particles_host(0, s)[0][0] for s in range(2)]
    step_and_compare(sim, p, prec, 4)
    tid1 = [sim.particles_host(0, s)[0][0] for s in range(2)]
    # both particles changed tile along both dimensions
    nt0 = 32 // 8
    for a, b in zip(tid0, tid1):
        assert a % nt0 != b % nt0 and a // nt0 != b // nt0, (a, b)
    sim.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_particles_start_on_faces(prec):
    """Positions on integer coordinates (cell faces, and tile faces at
    multiples of 8) in one or both dimensions, random momenta."""
    from paper_1906_06306_amd import _lib as L
    from paper_1906_06306_amd.sim import PicSim
    rng = np.random.default_rng(44)
    npart = 400
    xs, us = [], []
    for s in range(2):
        x = rng.uniform(0.0, 32.0, (2, npart))
        on = rng.integers(0, 3, npart)                 # 0: x on a face, 1: y, 2: both
        x[0, on != 1] = np.floor(x[0, on != 1])
        x[1, on != 0] = np.floor(x[1, on != 0])
        x[:, :40] = 8.0 * np.floor(x[:, :40] / 8.0)    # tile faces (and tile corners)
        xs.append(x)
        us.append(synth.sample_mj(rng, 0.3, npart))
    p = plasma_of(2, (32, 32), xs, us, 0.05, seed=45)
    print(f"[gpu] particles on faces, {prec}", flush=True)
    sim = PicSim(p, tile=(8, 8), precision=prec, capacity_factor=3.0, options=L.PIC_OPT_TRACK)
    step_and_compare(sim, p, prec, 2)
    sim.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_particles_at_rest_in_zero_fields(prec):
    from paper_1906_06306_amd import _lib as L
    from paper_1906_06306_amd.sim import PicSim
    rng = np.random.default_rng(46)
    npart = 300
    xs, us = [], []
    on_face = 0
    for s in range(2):
        x = rng.uniform(0.0, 24.0, (2, npart))
        x[0, : npart // 2] = np.floor(x[0, : npart // 2])   # half of them on an x face
        on_face += npart // 2
        xs.append(x)
        us.append(np.zeros((3, npart)))
    p = plasma_of(2, (24, 16), [xs[0][:, :], xs[1][:, :]], us, 0.0, seed=47)
    for sp in p.species:
        sp.x[1] = np.minimum(sp.x[1], 15.5)
    print(f"[gpu] particles at rest, {prec}", flush=True)
    sim = PicSim(p, tile=(8, 8), precision=prec, capacity_factor=2.0, options=L.PIC_OPT_TRACK)
    before = [sim.particles_host(0, s) for s in range(2)]
    sim.step(3, fused=True, half_b_in_push=True)
    assert sim.error() == 0
    E, B, J = sim.fields_host(0)
    assert not J.any() and not E.any() and not B.any()
    for s in range(2):
        t0, x0, u0 = before[s]
        t1, x1, u1 = sim.particles_host(0, s)
        # nothing moved: the same set of (tile, local position) pairs, u = 0
        a = sorted(zip(t0.tolist(), *[r.tolist() for r in x0]))
        b = sorted(zip(t1.tolist(), *[r.tolist() for r in x1]))
        assert a == b
        assert not u1.any()
    assert sim.diagnostics()["near_face"] == on_face
    sim.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_nonfinite_momentum_is_reported_and_contained(prec):
    """A particle whose four-velocity is NaN latches PIC_E_NONFINITE (read
    back, and cleared, by pic_error; latched again by the next step and
    then reported in the diagnostics' status), stays where it was and
    deposits nothing: the fields are the oracle's step of the other
    particles."""
    from paper_1906_06306_amd import _lib as L
    from paper_1906_06306_amd.sim import PicSim
    full = synth.small_random(2, (32, 24), 4, seed=48, field_amp=0.05)
    xs = [sp.x.copy() for sp in full.species]
    us = [sp.u.copy() for sp in full.species]
    us[0][:, 7] = np.nan
    p = plasma_of(2, (32, 24), xs, us, 0.05, seed=49)
    print(f"[gpu] NaN momentum, {p.nparticles} particles, {prec}", flush=True)
    sim = PicSim(p, tile=(8, 8), precision=prec, capacity_factor=3.0)
    sim.step(1, fused=True, half_b_in_push=True)
    err = sim.error()
    assert err & L.PIC_E_NONFINITE, err
    assert sim.error() == 0                         # read and cleared
    # the oracle's step without that particle
    q = plasma_of(2, (32, 24), [np.delete(xs[0], 7, axis=1), xs[1]], [np.delete(us[0], 7, axis=1), us[1]],
                  0.05, seed=49)
    st = oracle.State(q)
    st.step(1)
    E, B, J = sim.fields_host(0)
    tol = TOL[prec]
    assert rel(J, st.J) < tol and rel(E, st.E) < tol and rel(B, st.B) < tol
    tid, xl, u = sim.particles_host(0, 0)
    bad = ~np.isfinite(u).all(axis=0)
    assert bad.sum() == 1
    x_bad = tiles.to_global(tid[bad], xl[:, bad], (32, 24, 1), sim.T, 2)
    assert np.abs(x_bad[:, 0] - xs[0][:, 7]).max() < (1e-12 if prec == "fp64" else 4e-6)
    assert np.isfinite(sim.particles_host(0, 1)[2]).all()
    sim.step(1, fused=True, half_b_in_push=True)
    assert sim.diagnostics()["status"] & L.PIC_E_NONFINITE
    sim.close()


@pytest.mark.parametrize("prec", ["fp64"])
def test_cfl_violation_is_reported(prec):
    """At a Courant number of 1 (1D) a particle with u = 1e10 moves
    c u / gamma, a whole cell after rounding: PIC_E_CFL is latched and the
    particle is not moved; the slow particles step as in the oracle.  FP64
    only: there 1 + u^2 = 1e20 and its correctly rounded reciprocal square
    root give u / gamma = 1 exactly, while the FP32 push's reciprocal square
    root (about 1 ulp) may land either side of 1."""
    from paper_1906_06306_amd import _lib as L
    from paper_1906_06306_amd.sim import PicSim
    rng = np.random.default_rng(50)
    npart = 200
    xs = [rng.uniform(0.0, 64.0, (1, npart)) for _ in range(2)]
    us = [0.05 * rng.standard_normal((3, npart)) for _ in range(2)]
    us[1][:, 3] = (1e10, 0.0, 0.0)
    p = plasma_of(1, (64,), xs, us, 0.0, seed=51, c=1.0)
    print(f"[gpu] CFL violation, {p.nparticles} particles, c = 1, {prec}", flush=True)
    sim = PicSim(p, tile=(16,), precision=prec, capacity_factor=3.0)
    sim.step(1, fused=True, half_b_in_push=True)
    err = sim.error()
    assert err & L.PIC_E_CFL, err
    assert not err & L.PIC_E_NONFINITE
    tid, xl, u = sim.particles_host(0, 1)
    fast = u[0] > 1e9
    assert fast.sum() == 1
    xg = tiles.to_global(tid[fast], xl[:, fast], (64, 1, 1), sim.T, 1)
    assert abs(xg[0, 0] - xs[1][0, 3]) < (1e-12 if prec == "fp64" else 4e-6)
    q = plasma_of(1, (64,), [xs[0], np.delete(xs[1], 3, axis=1)], [us[0], np.delete(us[1], 3, axis=1)], 0.0,
                  seed=51, c=1.0)
    st = oracle.State(q)
    st.step(1)
    E, B, J = sim.fields_host(0)
    tol = TOL[prec]
    assert rel(J, st.J) < tol and rel(E, st.E) < tol
    sim.close()
