"""Pins of the oracle's other solvers from the paper's table of solvers: the
Vay and Higuera-Cary pushers and the 3-point binomial current filter, and of
the step that combines them (walls, pusher, filter passes).

* Pushers: with B = 0 all three give the exact electric kick; in a pure B
  they keep |u|; a particle in crossed fields moving at the force-free
  velocity (E + v x B = 0, here relativistic, gamma = 5) keeps its
  four-velocity to round-off with Vay and Higuera-Cary, which Boris does
  not; both converge at second order to the exact gyro-phase.
* Filter: a lattice Fourier mode is multiplied by prod_d cos^{2N}(k_d/2)
  after N passes (the binomial transfer function); the sum is kept.
* Step: with no option it equals orc_step (and with walls orc_step_walls)
  bit for bit; with N filter passes on the current, div E - F^N rho stays
  constant (the filter commutes with the lattice divergence).
"""
import math

import numpy as np
import pytest

import oracle
import synth

PUSHERS = {"boris": oracle.boris, "vay": oracle.vay, "hc": oracle.higuera_cary}


def one(v):
    return np.array(v, dtype=np.float64).reshape(3, 1)


@pytest.mark.parametrize("name", ["vay", "hc"])
def test_pure_electric_kick_equals_boris(name):
    rng = np.random.default_rng(1)
    u0 = rng.standard_normal((3, 50))
    E = rng.standard_normal((3, 50)) * 0.1
    B = np.zeros((3, 50))
    a, b = u0.copy(), u0.copy()
    oracle.boris(0.45, -1.0, E, B, a)
    PUSHERS[name](0.45, -1.0, E, B, b)
    assert np.abs(a - b).max() < 1e-15
    assert np.abs(b - (u0 - E / 0.45)).max() < 1e-14


@pytest.mark.parametrize("name", ["vay", "hc"])
def test_pure_magnetic_rotation_keeps_speed(name):
    rng = np.random.default_rng(2)
    u = rng.standard_normal((3, 100)) * 3
    B = rng.standard_normal((3, 100)) * 0.3
    E = np.zeros((3, 100))
    n0 = np.linalg.norm(u, axis=0)
    for _ in range(100):
        PUSHERS[name](0.45, 1.0, E, B, u)
    assert np.abs(np.linalg.norm(u, axis=0) - n0).max() < 1e-12 * n0.max()


def force_free_drift(name, steps=200):
    """Crossed fields E = -v x B with |v| = 0.9798 (gamma 5) along x."""
    c = 0.45
    gam = 5.0
    beta = math.sqrt(1 - 1 / gam ** 2)
    u = one([gam * beta, 0, 0])
    Bz = 0.2
    B = one([0, 0, Bz])
    # the Lorentz force per unit of s: E + (c v) x B / c with velocity in c
    # units is E + beta x B (App. C units), zero for E_y = beta B_z
    E = one([0, beta * Bz, 0])
    u0 = u.copy()
    for _ in range(steps):
        PUSHERS[name](c, 1.0, E, B, u)
    return np.abs(u - u0).max() / np.abs(u0).max()


@pytest.mark.parametrize("name", ["vay", "hc"])
def test_force_free_motion_is_kept(name):
    assert force_free_drift(name) < 1e-12


def test_boris_does_not_keep_force_free_motion():
    assert force_free_drift("boris") > 1e-4


def _gyro_phase_error(name, refine):
    """Phase of a relativistic gyration (gamma = 3) after a fixed time,
    time step refined by `refine` (c -> c / r, B -> B / r^2)."""
    c0, B0, T = 0.45, 0.3, 200
    c = c0 / refine
    B = B0 / refine ** 2
    steps = T * refine
    gam = 3.0
    up = math.sqrt(gam ** 2 - 1)
    u = one([up, 0, 0])
    E = np.zeros((3, 1))
    Bf = one([0, 0, B])
    for _ in range(steps):
        PUSHERS[name](c, 1.0, E, Bf, u)
    # exact rotation rate of u per step: s B / (gamma c) in these units
    omega = B / (gam * c)
    phase = math.atan2(u[1, 0], u[0, 0])
    exact = -omega * steps
    d = (phase - exact + math.pi) % (2 * math.pi) - math.pi
    return abs(d)


@pytest.mark.parametrize("name", ["vay", "hc"])
def test_second_order_gyro_phase(name):
    errs = [_gyro_phase_error(name, r) for r in (1, 2, 4, 8)]
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(3)]
    assert all(abs(o - 2.0) < 0.1 for o in orders), (errs, orders)


@pytest.mark.parametrize("D,n", [(1, (32,)), (2, (16, 12)), (3, (8, 6, 10))])
@pytest.mark.parametrize("passes", [1, 3, 8])
def test_binomial_transfer_function(D, n, passes):
    dims = tuple(n) + (1,) * (3 - D)
    N = int(np.prod(dims))
    idx = np.indices(dims[::-1]).reshape(3, -1)[::-1]   # (i, j, k) per cell, x fastest
    rng = np.random.default_rng(passes + D)
    m = [int(rng.integers(0, dims[d])) if d < D else 0 for d in range(3)]
    k = [2 * math.pi * m[d] / dims[d] for d in range(3)]
    F = np.cos(k[0] * idx[0] + k[1] * idx[1] + k[2] * idx[2] + 0.3)[None].repeat(3, axis=0).copy()
    F0 = F.copy()
    oracle.filter_binomial(D, n, passes, F)
    gain = np.prod([math.cos(k[d] / 2) ** (2 * passes) for d in range(D)])
    assert np.abs(F - gain * F0).max() < 1e-13
    G = rng.standard_normal((3, N))
    s0 = G.sum(axis=1)
    oracle.filter_binomial(D, n, passes, G)
    assert np.abs(G.sum(axis=1) - s0).max() < 1e-11


def opts_step(st, walls, pusher, passes):
    """One step through orc_step_opts (whatever the options)."""
    import ctypes
    from oracle import _dims, _p
    ns = len(st.x)
    dims = _dims(st.n)
    n_per = np.array([x.shape[1] for x in st.x], dtype=np.int64)
    xp = (ctypes.c_void_p * ns)(*[x.ctypes.data for x in st.x])
    up = (ctypes.c_void_p * ns)(*[u.ctypes.data for u in st.u])
    q = np.array(st.q)
    s = np.array(st.s)
    assert oracle.lib().orc_step_opts(st.D, _p(dims), st.c, ns, _p(n_per), ctypes.cast(xp, ctypes.c_void_p),
                                      ctypes.cast(up, ctypes.c_void_p), _p(q), _p(s), _p(st.E), _p(st.B),
                                      _p(st.J), walls, pusher, passes, 2) == 0


@pytest.mark.parametrize("walls", [False, True])
def test_option_step_reduces_to_plain_steps(walls):
    p = synth.small_random(2, (16, 12), 3, seed=4, theta=1.0, field_amp=0.05, q=0.01)
    a, b = oracle.State(p), oracle.State(p)
    if walls:
        a.hold_walls()
        b.hold_walls()
    for _ in range(3):
        a.step(1, walls=walls)
        opts_step(b, int(walls), 0, 0)
    assert all(np.array_equal(x, y) for x, y in zip(a.x, b.x))
    assert all(np.array_equal(x, y) for x, y in zip(a.u, b.u))
    assert np.array_equal(a.E, b.E) and np.array_equal(a.B, b.B) and np.array_equal(a.J, b.J)


@pytest.mark.parametrize("D,n,ppc", [(1, (32,), 16), (2, (16, 12), 4), (3, (8, 6, 6), 2)])
def test_filtered_gauss_law(D, n, ppc):
    """div E - F^N rho is constant when the current is filtered N times."""
    passes = 4
    p = synth.small_random(D, n, ppc, seed=8 + D, field_amp=0.02, q=0.01)
    st = oracle.State(p)

    def res():
        rho = st.rho()[None].copy()
        oracle.filter_binomial(D, n, passes, rho)
        return oracle.div_edge(st.n, st.E) - rho[0]
    r0 = res()
    for _ in range(10):
        st.step(1, pusher=2, filter_passes=passes)
    assert np.abs(res() - r0).max() < 1e-12


# ------------------------------------------------------------------ FDTD4

STAG = np.array([[0.5, 0, 0], [0, 0.5, 0], [0, 0, 0.5],
                 [0, 0.5, 0.5], [0.5, 0, 0.5], [0.5, 0.5, 0]])


def plane_wave4(D, n, c, m, e_dir, t):
    """Exact discrete plane wave of the fourth-order lattice: the staggered
    differences act as i kappa_d with kappa_d = 2 (9/8 sin(k_d/2) - 1/24
    sin(3 k_d/2)), so sin(w/2) = c |kappa| / 2 and B = c kappa x E /
    (2 sin(w/2)) (E at integer time t, B at t - 1/2)."""
    k = np.array([2 * math.pi * m[d] / n[d] if d < D else 0.0 for d in range(3)])
    kap = 2 * (9.0 / 8.0 * np.sin(k / 2) - 1.0 / 24.0 * np.sin(3 * k / 2))
    s = c * np.linalg.norm(kap) / 2
    w = 2 * math.asin(s)
    e = np.asarray(e_dir, float)
    e = e - kap * (e @ kap) / (kap @ kap)
    b = c * np.cross(kap, e) / (2 * s)
    N = n[0] * n[1] * n[2]
    cidx = np.arange(N)
    idx = np.stack([cidx % n[0], (cidx // n[0]) % n[1], cidx // (n[0] * n[1])]).astype(float)
    E = np.empty((3, N))
    B = np.empty((3, N))
    for comp in range(3):
        E[comp] = e[comp] * np.cos(k @ (idx + STAG[comp][:, None]) - w * t)
        B[comp] = b[comp] * np.cos(k @ (idx + STAG[3 + comp][:, None]) - w * (t - 0.5))
    return E, B


@pytest.mark.parametrize("D,n,m,e_dir", [
    (1, (32, 1, 1), (5, 0, 0), (0.0, 1.0, 0.5)),
    (2, (24, 16, 1), (3, 2, 0), (0.3, -0.2, 1.0)),
    (3, (16, 12, 10), (2, 3, 1), (0.7, -0.1, 0.4)),
])
def test_fdtd4_plane_wave_dispersion(D, n, m, e_dir):
    c = 0.45
    E, B = plane_wave4(D, n, c, m, e_dir, 0)
    for _ in range(1000):
        oracle.advance_b4(D, n, 0.5 * c, E, B)
        oracle.advance_b4(D, n, 0.5 * c, E, B)
        oracle.advance_e4(D, n, c, B, E)
    Ea, Ba = plane_wave4(D, n, c, m, e_dir, 1000)
    assert np.linalg.norm(E - Ea) / np.linalg.norm(Ea) < 1e-12
    assert np.linalg.norm(B - Ba) / np.linalg.norm(Ba) < 1e-12
    # the second-order lattice runs the same mode at another frequency
    E2, B2 = plane_wave4(D, n, c, m, e_dir, 0)
    for _ in range(200):
        oracle.advance_b(D, n, 0.5 * c, E2, B2)
        oracle.advance_b(D, n, 0.5 * c, E2, B2)
        oracle.advance_e(D, n, c, B2, E2)
    Ea, _ = plane_wave4(D, n, c, m, e_dir, 200)
    assert np.linalg.norm(E2 - Ea) / np.linalg.norm(Ea) > 1e-3


def div4(F, n, forward):
    """Fourth-order lattice divergence (same differences as the curls)."""
    nx, ny, nz = n
    G = F.reshape(3, nz, ny, nx)
    out = np.zeros((nz, ny, nx))
    for comp, ax in ((0, 2), (1, 1), (2, 0)):
        f = G[comp]
        if forward:
            out += 9 / 8 * (np.roll(f, -1, ax) - f) - 1 / 24 * (np.roll(f, -2, ax) - np.roll(f, 1, ax))
        else:
            out += 9 / 8 * (f - np.roll(f, 1, ax)) - 1 / 24 * (np.roll(f, -1, ax) - np.roll(f, 2, ax))
    return out.reshape(-1)


@pytest.mark.parametrize("D,n", [(2, (16, 12, 1)), (3, (8, 6, 10))])
def test_fdtd4_keeps_its_divergences(D, n):
    """div curl = 0 holds for the fourth-order differences taken with the
    same stencil: in vacuum, 10 steps keep the fourth-order div+ B and div- E
    of random fields.  (The first-order ZigZag current satisfies continuity
    with the second-order divergence, so with particles Gauss's law is exact
    only for FDTD2.)"""
    rng = np.random.default_rng(D)
    N = int(np.prod(n))
    E, B = rng.standard_normal((3, N)), rng.standard_normal((3, N))
    b0, e0 = div4(B, n, True), div4(E, n, False)
    for _ in range(10):
        oracle.advance_b4(D, n, 0.225, E, B)
        oracle.advance_b4(D, n, 0.225, E, B)
        oracle.advance_e4(D, n, 0.45, B, E)
    assert np.abs(div4(B, n, True) - b0).max() < 1e-12
    assert np.abs(div4(E, n, False) - e0).max() < 1e-12
