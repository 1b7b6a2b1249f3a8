"""Pins of the oracle's field solver (Eqs. fdE/fdB, App. B) against what
the discrete mathematics fixes: the Yee dispersion relation of an exact
discrete plane wave, the conserved leapfrog energy, and the divergence
identities div- curl- = div+ curl+ = 0."""
import math

import numpy as np
import pytest

# staggering offsets of Ex, Ey, Ez, Bx, By, Bz (main-text lattice, Sect. 2.3.1)
STAG = np.array([[0.5, 0, 0], [0, 0.5, 0], [0, 0, 0.5],
                 [0, 0.5, 0.5], [0.5, 0, 0.5], [0.5, 0.5, 0]])


def grid_index(n):
    N = n[0] * n[1] * n[2]
    c = np.arange(N)
    return np.stack([c % n[0], (c // n[0]) % n[1], c // (n[0] * n[1])]).astype(float)


def plane_wave(D, n, c, m, e_dir, t):
    """Exact discrete Yee plane wave: E at integer time t, B at t - 1/2.

    With kappa_d = 2 sin(k_d/2) the staggered differences act as i kappa,
    so a mode exp(i(k.x - w t)) needs sin(w/2) = c |kappa| / 2 and
    B = c kappa x E / (2 sin(w/2)) with E perpendicular to kappa."""
    k = np.array([2 * math.pi * m[d] / n[d] if d < D else 0.0 for d in range(3)])
    kap = 2 * np.sin(k / 2)
    s = c * np.linalg.norm(kap) / 2
    w = 2 * math.asin(s)
    e = np.asarray(e_dir, float)
    e = e - kap * (e @ kap) / (kap @ kap)
    b = c * np.cross(kap, e) / (2 * s)
    idx = grid_index(n)
    E = np.empty((3, idx.shape[1]))
    B = np.empty((3, idx.shape[1]))
    for comp in range(3):
        pos = idx + STAG[comp][:, None]
        E[comp] = e[comp] * np.cos(k @ pos - w * t)
        pos = idx + STAG[3 + comp][:, None]
        B[comp] = b[comp] * np.cos(k @ pos - w * (t - 0.5))
    return E, B


def vacuum_step(orc, D, n, c, E, B):
    orc.advance_b(D, n, 0.5 * c, E, B)   # push_half_b1
    orc.advance_b(D, n, 0.5 * c, E, B)   # push_half_b2
    orc.advance_e(D, n, c, B, E)         # push_e


@pytest.mark.parametrize("D,n,m,e_dir", [
    (1, (32, 1, 1), (3, 0, 0), (0.0, 1.0, 0.5)),
    (2, (24, 16, 1), (2, 1, 0), (0.3, -0.2, 1.0)),
    (2, (24, 16, 1), (1, 3, 0), (1.0, 0.4, 0.0)),
    (3, (16, 12, 10), (1, 2, 1), (0.7, -0.1, 0.4)),
    (3, (10, 14, 12), (2, 1, 3), (-0.2, 0.9, 0.3)),
])
def test_vacuum_plane_wave_dispersion(orc, D, n, m, e_dir):
    """P-1: 1000 steps of the split-B FDTD reproduce the exact discrete
    plane wave (Yee dispersion sin^2(w/2) = c^2 sum sin^2(k/2))."""
    c = 0.45
    E, B = plane_wave(D, n, c, m, e_dir, 0)
    steps = 1000
    for _ in range(steps):
        vacuum_step(orc, D, n, c, E, B)
    Ea, Ba = plane_wave(D, n, c, m, e_dir, steps)
    err_e = np.linalg.norm(E - Ea) / np.linalg.norm(Ea)
    err_b = np.linalg.norm(B - Ba) / np.linalg.norm(Ba)
    assert err_e < 1e-12 and err_b < 1e-12, (err_e, err_b)


def test_plane_wave_detects_wrong_dispersion(orc):
    """The pin is sharp: after 200 steps the continuum dispersion w = c|k|
    is off by far more than the tolerance, so a stencil error that moved the
    numerical frequency would be caught."""
    D, n, c, m = 2, (24, 16, 1), 0.45, (2, 1, 0)
    e_dir = (0.3, -0.2, 1.0)
    E, B = plane_wave(D, n, c, m, e_dir, 0)
    for _ in range(200):
        vacuum_step(orc, D, n, c, E, B)
    Ea, _ = plane_wave(D, n, c, m, e_dir, 200)
    assert np.linalg.norm(E - Ea) / np.linalg.norm(Ea) < 1e-12
    k = np.array([2 * math.pi * 2 / 24, 2 * math.pi / 16, 0.0])
    w_disc = 2 * math.asin(c * np.linalg.norm(2 * np.sin(k / 2)) / 2)
    w_cont = c * np.linalg.norm(k)
    idx = grid_index(n)
    ez_cont = np.cos(k @ (idx + STAG[2][:, None]) - w_cont * 200)
    ez_disc = np.cos(k @ (idx + STAG[2][:, None]) - w_disc * 200)
    assert np.abs(ez_cont - ez_disc).max() > 1e-3


@pytest.mark.parametrize("D,n", [(1, (40, 1, 1)), (2, (20, 14, 1)), (3, (10, 8, 6))])
def test_vacuum_energy_and_divergence(orc, D, n):
    """P-2: 1/2 sum(E^n.E^n + B^(n-1/2).B^(n+1/2)) is exactly conserved by the
    leapfrog in vacuum (curl- is the adjoint of curl+ on a periodic grid),
    and div+ B and div- E do not change."""
    rng = np.random.default_rng(7)
    c = 0.45
    N = n[0] * n[1] * n[2]
    E = rng.standard_normal((3, N))
    B = rng.standard_normal((3, N))
    inv = []
    for _ in range(300):
        Bp = B.copy()
        orc.advance_b(D, n, c, E, Bp)          # B^{n+1/2} from B^{n-1/2}
        inv.append(0.5 * (np.sum(E * E) + np.sum(B * Bp)))
        vacuum_step(orc, D, n, c, E, B)
    inv = np.array(inv)
    assert np.abs(inv - inv[0]).max() < 1e-12 * abs(inv[0])
    E2 = rng.standard_normal((3, N))
    B2 = rng.standard_normal((3, N))
    divb0 = orc.div_face(n, B2)
    dive0 = orc.div_edge(n, E2)
    for _ in range(100):
        vacuum_step(orc, D, n, c, E2, B2)
    assert np.abs(orc.div_face(n, B2) - divb0).max() < 1e-12
    assert np.abs(orc.div_edge(n, E2) - dive0).max() < 1e-12


def test_curl_adjointness(orc):
    """sum B.(curl+ E) == sum E.(curl- B) on a periodic 3D grid: the two
    difference stencils are transposes of each other (App. B)."""
    rng = np.random.default_rng(3)
    n = (7, 5, 6)
    N = 7 * 5 * 6
    E = rng.standard_normal((3, N))
    B = rng.standard_normal((3, N))
    Z = np.zeros((3, N))
    cE = Z.copy()
    orc.advance_b(3, n, -1.0, E, cE)            # cE = +curl+ E
    cB = Z.copy()
    orc.advance_e(3, n, 1.0, B, cB)             # cB = curl- B
    assert abs(np.sum(B * cE) - np.sum(E * cB)) < 1e-11


def test_add_current(orc):
    n = (4, 3, 2)
    E = np.ones((3, 24))
    J = np.arange(72, dtype=float).reshape(3, 24)
    orc.add_current(n, J, E)
    assert np.array_equal(E, 1.0 - J)
