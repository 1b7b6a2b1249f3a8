"""Pins of the oracle's conducting, reflecting walls in x (the shock
configuration's boundary; y and z stay periodic).

* A vacuum standing wave between the walls, Ey = sin(k i) with k = m pi/n0,
  follows the closed form of the discrete Yee lattice, cos(omega n) with
  sin(omega/2) = c sin(k/2), for odd m too, where the periodic lattice
  cannot hold it.
* A lone particle that crosses a wall comes back mirrored (x -> -x or
  2 n0 - x, u_x -> -u_x).
* Charge conservation: with particles bouncing off both walls, Gauss's
  residual div E - rho stays constant to round-off at every node off the
  wall plane (the broken-path ZigZag deposit keeps continuity exact).
* The wall planes stay at zero tangential E and normal B.
"""
import math

import numpy as np
import pytest

import oracle
import synth


def standing_wave_state(D, n, m, c=0.45):
    p = synth.small_random(D, n, 1, seed=1)
    for sp in p.species:
        sp.x = sp.x[:, :0].copy()
        sp.u = sp.u[:, :0].copy()
    st = oracle.State(p)
    st.E[:] = 0.0
    st.B[:] = 0.0
    N = int(np.prod(st.n))
    i = np.arange(N) % n[0]
    k = m * math.pi / n[0]
    w = 2.0 * math.asin(c * math.sin(0.5 * k))
    st.E[1] = np.sin(k * i)
    # B^{-1/2} at i+1/2: -cos(k(i+1/2)) sin(omega (n+1/2)) at n = -1
    st.B[2] = math.sin(0.5 * w) * np.cos(k * (i + 0.5))
    return st, k, w, i


@pytest.mark.parametrize("D,n", [(1, (24,)), (2, (20, 6))])
@pytest.mark.parametrize("m", [1, 2, 3])
def test_standing_wave_between_walls(D, n, m):
    st, k, w, i = standing_wave_state(D, n, m)
    nsteps = 37
    st.step(nsteps, walls=True)
    assert np.abs(st.E[1] - np.sin(k * i) * math.cos(w * nsteps)).max() < 1e-12
    # after N steps the state holds B^{N-1/2}
    bz = -np.cos(k * (i + 0.5)) * math.sin(w * (nsteps - 0.5))
    assert np.abs(st.B[2] - bz).max() < 1e-12
    assert np.abs(st.E[0]).max() == 0.0 and np.abs(st.E[2]).max() == 0.0


def test_periodic_lattice_cannot_hold_odd_standing_wave():
    st, k, w, i = standing_wave_state(1, (24,), 1)
    st.step(37)
    assert np.abs(st.E[1] - np.sin(k * i) * math.cos(w * 37)).max() > 1e-3


@pytest.mark.parametrize("side", ["left", "right"])
def test_single_particle_reflects(side):
    n = (16, 8)
    p = synth.small_random(2, n, 1, seed=2, field_amp=0.0, q=1e-9)
    for sp in p.species:
        sp.x = sp.x[:, :1].copy()
        sp.u = sp.u[:, :1].copy()
    ux = 2.0
    if side == "left":
        p.species[0].x[:, 0] = [0.1, 3.3]
        p.species[0].u[:, 0] = [-ux, 0.5, 0.2]
    else:
        p.species[0].x[:, 0] = [15.9, 3.3]
        p.species[0].u[:, 0] = [ux, 0.5, 0.2]
    p.species[1].x[:, 0] = [8.0, 4.0]
    p.species[1].u[:, 0] = [0.0, 0.0, 0.0]
    st = oracle.State(p)
    x0 = st.x[0][:, 0].copy()
    u0 = st.u[0][:, 0].copy()
    st.step(1, walls=True)
    g = math.sqrt(1.0 + (u0 ** 2).sum())
    dx = st.c * u0[:2] / g
    free = x0 + dx
    want_x = -free[0] if side == "left" else 2 * n[0] - free[0]
    assert abs(st.x[0][0, 0] - want_x) < 1e-12
    assert abs(st.x[0][1, 0] - free[1]) < 1e-12
    assert abs(st.u[0][0, 0] + u0[0]) < 1e-9 * abs(u0[0])


@pytest.mark.parametrize("D,n,ppc", [(1, (32,), 16), (2, (16, 12), 4), (3, (8, 6, 6), 2)])
def test_charge_conservation_with_walls(D, n, ppc):
    """Gauss residual constant at every node off the wall plane over 30
    steps of a hot plasma that keeps hitting both walls."""
    p = synth.small_random(D, n, ppc, theta=2.0, seed=5 + D, field_amp=0.0, q=0.01)
    st = oracle.State(p)
    st.hold_walls()
    N = int(np.prod(st.n))
    interior = (np.arange(N) % n[0]) != 0
    r0 = st.gauss_residual()
    flips = 0
    for _ in range(30):
        ux = [u[0].copy() for u in st.u]
        st.step(1, walls=True)
        flips += sum(int((np.sign(a) != np.sign(u[0])).sum()) for a, u in zip(ux, st.u))
        r = st.gauss_residual()
        assert np.abs(r - r0)[interior].max() < 1e-12
        for x in st.x:
            assert x[0].min() >= 0.0 and x[0].max() < n[0]
    assert flips > 10
    idx = np.arange(0, N, n[0])
    assert not st.E[1, idx].any() and not st.E[2, idx].any() and not st.B[0, idx].any()


def test_interpolation_images_at_walls():
    """Half-integer components mirror (value at -1/2 = value at +1/2, at
    n0+1/2 = at n0-1/2); node components vanish on the wall planes."""
    D, n = 2, (10, 4)
    N = 40
    i = np.arange(N) % n[0]
    E = np.zeros((3, N))
    B = np.zeros((3, N))
    E[0] = 1.0 + 0.1 * i       # Ex at i+1/2
    E[1] = 2.0 + 0.3 * i       # Ey at node i (i = 0 is the wall plane)
    B[1] = -1.0 + 0.2 * i      # By at i+1/2
    B[0] = 0.5 + 0.05 * i      # Bx at node i
    E[1, i == 0] = 0.0
    B[0, i == 0] = 0.0
    x = np.array([[0.2, 9.8, 0.7, 9.3], [1.0, 1.0, 1.0, 1.0]])
    Ep, Bp = oracle.interp(D, n, E, B, x, walls=True)
    # Ex: x=0.2 lies between the image at -1/2 and +1/2 (equal values)
    assert abs(Ep[0, 0] - 1.0) < 1e-15
    assert abs(Ep[0, 1] - (1.0 + 0.1 * 9)) < 1e-15
    assert abs(Bp[1, 0] - (-1.0)) < 1e-15 and abs(Bp[1, 1] - (-1.0 + 0.2 * 9)) < 1e-15
    # Ey, Bx at x = 9.8: (1-w) value(9) + w * 0 (the wall node n0)
    assert abs(Ep[1, 1] - 0.2 * (2.0 + 0.3 * 9)) < 1e-14
    assert abs(Bp[0, 1] - 0.2 * (0.5 + 0.05 * 9)) < 1e-14
    # interior points agree with the periodic interpolation
    Eq, Bq = oracle.interp(D, n, E, B, x[:, 2:], walls=False)
    assert np.abs(Eq - Ep[:, 2:]).max() < 1e-15 and np.abs(Bq - Bp[:, 2:]).max() < 1e-15
