"""Particle creation in tiles (pic_inject) with the receding-wall injector
of the shock setup: injected particles are binned bit-exactly like the
initial ones (appended after a tile's particles, input order kept), and a
run that starts from an empty upstream and injects a slab every step
matches the oracle fed the same slabs (FP64, 1e-12 after each step; FP32,
1e-5 after one step), with Gauss's law kept (pairs are injected on top of
each other)."""
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


def setup(D, n, T, prec, walls):
    from paper_1906_06306_amd.sim import PicSim
    if D == 3:
        p = synth.shock(n=n, x_shock=n[0] // 4)
    else:
        # hot pairs in the left quarter, vacuum to the right of the injector
        rng = np.random.default_rng(5)
        x = synth.quiet_positions(rng, 2, (n[0] // 4, n[1], 1), 2)
        q = 1.2656e-3
        sp = [synth.Species(-q, -1.0, q, x.copy(), synth.sample_mj(rng, 1.0, x.shape[1])),
              synth.Species(q, 1.0, q, x.copy(), synth.sample_mj(rng, 1.0, x.shape[1]))]
        N = n[0] * n[1]
        p = synth.Plasma(D=2, n=n, c=0.45, species=sp, E=np.zeros((3, N)), B=np.zeros((3, N)))
    inj = synth.RecedingInjector(n[:D], ppc=4, gamma=10.0, theta=1e-4, c=p.c, x0=float(n[0] // 4))
    tcap = "auto"
    print(f"[gpu] inject D={D} n={n} T={T} {prec} walls={walls}", flush=True)
    sim = PicSim(p, tile=T[:D], precision=prec, walls=walls, tile_capacity=tcap, capacity_factor=3.0,
                 inject_max=200000)
    return p, inj, sim


@pytest.mark.parametrize("D,n,T", [(2, (64, 16, 1), (8, 8, 1)), (3, (32, 8, 8), (8, 4, 4))])
def test_injected_particles_bin_like_initial_ones(D, n, T):
    p, inj, sim = setup(D, n, T, "fp32", True)
    before = [sim.particles_host(0, s) for s in range(2)]
    x, ue, up = inj.batch(0)
    sim.inject(0, 0, x, ue)
    sim.inject(0, 1, x, up)
    assert sim.error() == 0
    for s, u_new in ((0, ue), (1, up)):
        tid0, xl0, u0 = before[s]
        tid1, xl1, u1 = sim.particles_host(0, s)
        t_new, xl_new, order = tiles.bin_global(x, n, T, D, np.float32, walls=True)
        # expected: per tile, the old particles, then the new ones in input order
        exp_t = np.concatenate([tid0, t_new])
        exp_x = np.concatenate([xl0, xl_new], axis=1)
        exp_u = np.concatenate([u0, u_new.astype(np.float32)], axis=1)
        o = np.argsort(exp_t, kind="stable")
        assert np.array_equal(tid1, exp_t[o])
        assert np.array_equal(xl1, exp_x[:, o]) and np.array_equal(u1, exp_u[:, o])
    sim.close()


@pytest.mark.parametrize("prec,steps,tol", [("fp64", 6, 1e-12), ("fp32", 1, 1e-5)])
@pytest.mark.parametrize("D,n,T", [(2, (64, 16, 1), (8, 8, 1)), (3, (32, 8, 8), (8, 4, 4))])
def test_receding_injector_run_matches_oracle(D, n, T, prec, steps, tol):
    p, inj, sim = setup(D, n, T, prec, True)
    st = oracle.State(p)
    E, B, _ = sim.fields_host(0)
    st.E[:] = E
    st.B[:] = B
    for s in range(2):
        tid, xl, u = sim.particles_host(0, s)
        st.x[s] = np.ascontiguousarray(tiles.to_global(tid, xl, n, T, D))
        st.u[s] = np.ascontiguousarray(u.astype(np.float64))
    st.hold_walls()
    g0 = st.gauss_residual()
    for k in range(steps):
        x, ue, up = inj.batch(k)
        sim.inject(0, 0, x, ue)
        sim.inject(0, 1, x, up)
        x32 = x if prec == "fp64" else None
        if prec == "fp32":
            # the oracle takes what the GPU stored (tile-local FP32 widened)
            st2 = []
            for s in range(2):
                tid, xl, u = sim.particles_host(0, s)
                st.x[s] = np.ascontiguousarray(tiles.to_global(tid, xl, n, T, D))
                st.u[s] = np.ascontiguousarray(u.astype(np.float64))
        else:
            st.append(0, x32, ue)
            st.append(1, x32, up)
        sim.step(1, fused=True, half_b_in_push=True)
        st.step(1, walls=True)
        assert sim.error() == 0
        E, B, J = sim.fields_host(0)
        assert rel(J, st.J) < tol and rel(E, st.E) < tol and rel(B, st.B) < tol, (k, rel(J, st.J), rel(E, st.E))
    d = sim.diagnostics()
    assert d["particles"] == sum(x.shape[1] for x in st.x)
    if prec == "fp64":
        interior = (np.arange(g0.size) % n[0]) != 0
        assert np.abs(st.gauss_residual() - g0)[interior].max() < 1e-12
    sim.close()
