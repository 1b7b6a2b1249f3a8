"""Pins of the oracle's particle routines against closed forms, invariants
and brute force: linear interpolation (Sect. 2.3.2), the relativistic Boris
update (App. C), the position advance (Eq. fdX) and the ZigZag deposit
(App. D)."""
import math

import numpy as np
import pytest

STAG = np.array([[0.5, 0, 0], [0, 0.5, 0], [0, 0, 0.5],
                 [0, 0.5, 0.5], [0.5, 0, 0.5], [0.5, 0.5, 0]])


def grid_index(n):
    N = n[0] * n[1] * n[2]
    c = np.arange(N)
    return np.stack([c % n[0], (c // n[0]) % n[1], c // (n[0] * n[1])]).astype(float)


# ----------------------------------------------------------- interpolation

@pytest.mark.parametrize("D", [1, 2, 3])
def test_interp_constant_and_linear_fields(orc, D):
    """P-3: constant fields and fields linear in position along each
    component's own staggered lattice are reproduced exactly at arbitrary
    positions (away from the periodic seam)."""
    n = tuple([12] * D + [1] * (3 - D))
    N = int(np.prod(n))
    rng = np.random.default_rng(11)
    a = rng.standard_normal(6)
    g = rng.standard_normal((6, 3))
    g[:, D:] = 0.0
    idx = grid_index(n)
    F = np.empty((6, N))
    for comp in range(6):
        pos = idx + STAG[comp][:, None]
        F[comp] = a[comp] + g[comp] @ pos
    x = rng.uniform(2.0, 9.0, (D, 500))
    Ep, Bp = orc.interp(D, n, F[:3].copy(), F[3:].copy(), x)
    xx = np.zeros((3, 500))
    xx[:D] = x
    want = a[:, None] + g @ xx
    assert np.abs(Ep - want[:3]).max() < 1e-12
    assert np.abs(Bp - want[3:]).max() < 1e-12
    C = np.tile(a[:, None], (1, N))
    Ep, Bp = orc.interp(D, n, C[:3].copy(), C[3:].copy(), rng.uniform(0, 12, (D, 300)))
    assert np.abs(Ep - a[:3, None]).max() < 1e-14
    assert np.abs(Bp - a[3:, None]).max() < 1e-14


def test_interp_lattice_points(orc):
    """A particle sitting on a component's own lattice point reads exactly
    that stored value (weights 1, 0, ...)."""
    n = (8, 8, 8)
    rng = np.random.default_rng(5)
    E = rng.standard_normal((3, 512))
    B = rng.standard_normal((3, 512))
    i, j, k = 3, 5, 2
    c = i + 8 * (j + 8 * k)
    for comp in range(6):
        x = (np.array([i, j, k], float) + STAG[comp])[:, None]
        Ep, Bp = orc.interp(3, n, E, B, x)
        got = Ep[comp, 0] if comp < 3 else Bp[comp - 3, 0]
        want = E[comp, c] if comp < 3 else B[comp - 3, c]
        assert got == want


# ------------------------------------------------------------------ Boris

def run_push(orc, c, s, Evec, Bvec, u0, x0, steps):
    """Single particle in uniform fields; returns u (steps+1, 3) and x."""
    u = np.array(u0, float).reshape(3, 1).copy()
    x = np.array(x0, float).reshape(3, 1).copy()
    Ep = np.array(Evec, float).reshape(3, 1)
    Bp = np.array(Bvec, float).reshape(3, 1)
    us = [u[:, 0].copy()]
    xs = [x[:, 0].copy()]
    for _ in range(steps):
        orc.boris(c, s, Ep, Bp, u)
        orc.move(3, c, u, x)
        us.append(u[:, 0].copy())
        xs.append(x[:, 0].copy())
    return np.array(us), np.array(xs)


@pytest.mark.parametrize("s", [1.0, -1.0])
def test_boris_pure_b_gyration(orc, s):
    """P-4: in a uniform B, |u| is conserved, the rotation angle per step is
    exactly 2 arctan(|s|B/(2 c gamma)) (sense set by sign(s B)), and the
    positions are the vertices of a regular polygon of circumradius
    r_L sqrt(1+t^2), r_L = c^2 |u_perp| / (|s| B)."""
    c, Bz = 0.45, 0.2
    u0 = np.array([0.5, -0.2, 0.3])
    steps = 10000
    us, xs = run_push(orc, c, s, (0, 0, 0), (0, 0, Bz), u0, (0, 0, 0), steps)
    g = math.sqrt(1 + u0 @ u0)
    mag = np.sqrt((us ** 2).sum(1))
    assert np.abs(mag - mag[0]).max() < 1e-13
    t = abs(s) * Bz / (2 * c * g)
    th = -np.sign(s * Bz) * 2 * math.atan(t)
    nn = np.arange(steps + 1)
    ph = np.arctan2(u0[1], u0[0]) + nn * th
    uperp = math.hypot(u0[0], u0[1])
    want = np.stack([uperp * np.cos(ph), uperp * np.sin(ph)], 1)
    assert np.abs(us[:, :2] - want).max() < 1e-11 * uperp
    assert np.abs(us[:, 2] - u0[2]).max() < 1e-14
    R = c * c * uperp * math.sqrt(1 + t * t) / (abs(s) * Bz)
    # circumcentre from the first three vertices
    p0, p1, p2 = xs[0, :2], xs[1, :2], xs[2, :2]
    A = 2 * np.array([p1 - p0, p2 - p0])
    rhs = np.array([p1 @ p1 - p0 @ p0, p2 @ p2 - p0 @ p0])
    ctr = np.linalg.solve(A, rhs)
    dist = np.sqrt(((xs[:, :2] - ctr) ** 2).sum(1))
    assert abs(dist[0] - R) < 1e-12 * R
    assert np.abs(dist - R).max() < 1e-9 * R
    # parallel motion: uniform, c u_z / gamma per step
    assert abs(xs[-1, 2] - steps * c * u0[2] / g) < 1e-9


@pytest.mark.parametrize("s", [1.0, -1.0])
def test_boris_pure_e_kick(orc, s):
    """P-5: with B = 0, every step adds exactly s E / c to u."""
    c = 0.45
    E = np.array([0.01, -0.02, 0.005])
    u0 = np.array([0.1, 0.0, -0.3])
    us, _ = run_push(orc, c, s, E, (0, 0, 0), u0, (0, 0, 0), 500)
    want = u0[None, :] + np.arange(501)[:, None] * (s * E / c)[None, :]
    assert np.abs(us - want).max() < 1e-12


def test_boris_exb_drift(orc):
    """P-6: in crossed fields with |E|/|B| = 0.05 and w_B dt <= 0.1 the mean
    velocity over many gyro-periods tends to c E x B / B^2 (cells/step)."""
    c, Bz, Ey = 0.45, 0.045, 0.05 * 0.045
    us, xs = run_push(orc, c, 1.0, (0, Ey, 0), (0, 0, Bz), (0, 0, 0), (0, 0, 0), 63000)
    vd = c * np.cross([0, Ey, 0], [0, 0, Bz]) / Bz ** 2
    vmean = (xs[-1] - xs[0]) / (len(xs) - 1)
    assert abs(vmean[0] - vd[0]) < 1e-3 * abs(vd[0])
    assert abs(vmean[1]) < 1e-3 * abs(vd[0]) and abs(vmean[2]) < 1e-15


def _hyperbolic_error(orc, refine):
    """Position error at fixed physical time for uniform E along x,
    starting at rest; time step refined by `refine` (c -> c/r, E -> E/r^2)."""
    c0, E0, T = 0.45, 0.02, 200
    c = c0 / refine
    E = E0 / refine ** 2
    steps = T * refine
    _, xs = run_push(orc, c, 1.0, (E, 0, 0), (0, 0, 0), (0, 0, 0), (0, 0, 0), steps)
    a = E / c                 # u^{n+1/2} = u^{n-1/2} + a, with u^{-1/2} = 0
    # continuous: u(t) = a (t + 1/2) measured in steps, x = c/a (gamma(t) - gamma(0))
    t = steps
    x_exact = (c / a) * (math.sqrt(1 + (a * (t + 0.5)) ** 2) - math.sqrt(1 + (a * 0.5) ** 2))
    return abs(xs[-1, 0] - x_exact)


def _gyro_phase_error(orc, refine):
    c0, B0, T = 0.45, 0.3, 300
    c = c0 / refine
    B = B0 / refine ** 2
    steps = T * refine
    u0 = np.array([1.0, 0.0, 0.0])
    us, _ = run_push(orc, c, 1.0, (0, 0, 0), (0, 0, B), u0, (0, 0, 0), steps)
    g = math.sqrt(2.0)
    w = B / (c * g)           # exact continuous angle per step
    ph = math.atan2(us[-1, 1], us[-1, 0])
    want = -w * steps
    d = (ph - want + math.pi) % (2 * math.pi) - math.pi
    return abs(d)


@pytest.mark.parametrize("errfn", [_hyperbolic_error, _gyro_phase_error])
def test_boris_second_order_convergence(orc, errfn):
    """P-13: errors against exact continuous orbits (hyperbolic motion in a
    uniform E; gyro-phase in a uniform B) fall as the square of the step."""
    errs = [errfn(orc, r) for r in (1, 2, 4, 8)]
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(3)]
    assert all(abs(o - 2.0) < 0.1 for o in orders), (errs, orders)


def test_move_uses_updated_gamma(orc):
    """Eq. fdX: dx = c u/gamma with gamma of the same u, all 3 components."""
    u = np.array([[2.0], [-2.0], [4.0]])       # gamma = sqrt(1 + 24) = 5
    x = np.array([[1.0], [2.0]])
    disp = orc.move(2, 0.45, u, x)
    assert np.allclose(disp[:, 0], 0.45 * np.array([2.0, -2.0, 4.0]) / 5.0, rtol=0, atol=1e-16)
    assert np.allclose(x[:, 0], [1.0 + disp[0, 0], 2.0 + disp[1, 0]], rtol=0, atol=0)


# ----------------------------------------------------------------- ZigZag

def _continuity(orc, D, n, q, x1, x2, disp):
    N = int(np.prod(n))
    J = np.zeros((3, N))
    orc.zigzag(D, n, q, x1, x2, disp, J)
    r = orc.rho(D, n, q, x2) - orc.rho(D, n, q, x1) + orc.div_edge(n, J)
    return r, J


@pytest.mark.parametrize("D", [1, 2, 3])
def test_zigzag_continuity_brute_force(orc, D):
    """P-7: rho^{n+1} - rho^n + div- J = 0 on every node for random
    displacements |dx_d| < 1, including moves that start within 1e-12 of a
    cell face and cross it; 1e6 displacements per dimension in 1000
    batches of 1000 particles on a 16^D periodic grid."""
    n = tuple([16] * D + [1] * (3 - D))
    rng = np.random.default_rng(100 + D)
    q = 0.37
    worst = 0.0
    batches = 1000 if D < 3 else 250
    per = 1000 if D < 3 else 4000
    for b in range(batches):
        x1 = rng.uniform(0, 16, (D, per))
        if b % 4 == 0:   # start right at a face, move across it
            x1 = np.floor(x1) + rng.choice([1e-12, 1 - 1e-12, 0.0], size=(D, per))
        disp = rng.uniform(-0.999, 0.999, (3, per))
        x2 = x1 + disp[:D]
        r, _ = _continuity(orc, D, n, q, x1, x2, disp)
        worst = max(worst, np.abs(r).max())
    assert worst < 1e-14 * q * 16, worst


def test_zigzag_continuity_catches_missing_3d_term(orc):
    """The continuity pin is sharp in 3D: a deposit that keeps the
    App. D relay point, fluxes and midpoint weights but drops the
    path-average dv_a dv_b/12 term (built here independently in numpy)
    leaves an O(dy dz/48) residual, while the oracle's residual is round-off."""
    n = (6, 6, 6)
    x1 = np.array([2.3, 2.6, 2.1])
    d = np.array([0.6, 0.7, -0.8])
    x2 = x1 + d
    r, _ = _continuity(orc, 3, n, 1.0, x1[:, None], x2[:, None], d[:, None])
    assert np.abs(r).max() < 1e-15
    i1, i2 = np.floor(x1), np.floor(x2)
    xr = np.minimum(np.minimum(i1, i2) + 1, np.maximum(np.maximum(i1, i2), 0.5 * (x1 + x2)))
    J = np.zeros((3, 6, 6, 6))     # [comp, k, j, i]
    for F, W, ii in ((xr - x1, 0.5 * (x1 + xr) - i1, i1), (x2 - xr, 0.5 * (x2 + xr) - i2, i2)):
        ii = ii.astype(int)
        for m in range(3):
            a_, b_ = [dd for dd in range(3) if dd != m]
            for ca in (0, 1):
                for cb in (0, 1):
                    idx = ii.copy()
                    idx[a_] += ca
                    idx[b_] += cb
                    w = (W[a_] if ca else 1 - W[a_]) * (W[b_] if cb else 1 - W[b_])
                    J[m, idx[2] % 6, idx[1] % 6, idx[0] % 6] += F[m] * w
    r2 = (orc.rho(3, n, 1.0, x2[:, None]) - orc.rho(3, n, 1.0, x1[:, None])
          + orc.div_edge(n, J.reshape(3, -1)))
    assert np.abs(r2).max() > 1e-3


def test_zigzag_sum_rule_and_antisymmetry(orc):
    """P-8: sum over cells of J_m equals q dx_m for every particle (the two
    fluxes add up to the displacement and the weights sum to one), and
    reversing the move reverses the current exactly."""
    rng = np.random.default_rng(21)
    for D in (1, 2, 3):
        n = tuple([8] * D + [1] * (3 - D))
        N = int(np.prod(n))
        for _ in range(200):
            x1 = rng.uniform(1, 7, (D, 1))
            d = rng.uniform(-0.99, 0.99, (3, 1))
            x2 = x1 + d[:D]
            J = np.zeros((3, N))
            orc.zigzag(D, n, 0.5, x1, x2, d, J)
            assert np.allclose(J.sum(1), 0.5 * d[:, 0], rtol=0, atol=1e-15)
            Jr = np.zeros((3, N))
            orc.zigzag(D, n, 0.5, x2, x1, -d, Jr)
            assert np.abs(J + Jr).max() < 1e-15


def test_zigzag_same_cell_is_villasenor_buneman(orc):
    """A move inside one cell: the in-plane current equals the classic
    area-weighting (Villasenor-Buneman) current of the straight path,
    Jx(i+1/2, j) = q dx (1 - y_mid), Jx(i+1/2, j+1) = q dx y_mid, and
    likewise for Jy."""
    n = (8, 8, 1)
    x1 = np.array([[3.2], [4.3]])
    d = np.array([[0.5], [0.4], [0.0]])
    x2 = x1 + d[:2]
    J = np.zeros((3, 64))
    orc.zigzag(2, n, 1.0, x1, x2, d, J)
    xm, ym = 3.45 - 3, 4.5 - 4
    Jx = J[0].reshape(8, 8)
    Jy = J[1].reshape(8, 8)
    assert abs(Jx[4, 3] - 0.5 * (1 - ym)) < 1e-15 and abs(Jx[5, 3] - 0.5 * ym) < 1e-15
    assert abs(Jy[4, 3] - 0.4 * (1 - xm)) < 1e-15 and abs(Jy[4, 4] - 0.4 * xm) < 1e-15
    assert abs(J[0].sum() - 0.5) < 1e-15 and np.count_nonzero(J[0]) == 2


def test_zigzag_face_crossing_relay(orc):
    """A 1D move from 1.8 to 2.3 crosses the face at 2: the relay point sits
    on the face, so 0.2 q goes through J at 1+1/2 and 0.3 q at 2+1/2.  In 1D
    the current is unique (continuity plus the sum rule fix it)."""
    n = (6, 1, 1)
    J = np.zeros((3, 6))
    orc.zigzag(1, n, 1.0, np.array([[1.8]]), np.array([[2.3]]), np.array([[0.5], [0], [0]]), J)
    assert np.allclose(J[0], [0, 0.2, 0.3, 0, 0, 0], rtol=0, atol=1e-15)


def test_zigzag_out_of_plane_only(orc):
    """No in-plane motion: J_z is q dz times the cloud-in-cell weights of the
    position (2D), which is the charge-density stencil."""
    n = (6, 6, 1)
    x = np.array([[2.25], [3.5]])
    d = np.array([[0.0], [0.0], [0.3]])
    J = np.zeros((3, 36))
    orc.zigzag(2, n, 2.0, x, x.copy(), d, J)
    rho = orc.rho(2, n, 1.0, x)
    assert np.abs(J[2] - 2.0 * 0.3 * rho).max() < 1e-15
    assert np.abs(J[:2]).max() == 0.0


# ------------------------------------------------------------ Langmuir

def test_langmuir_frequency_pins_units(orc):
    """P-10: cold pair plasma, uniform (k=0) counter-motion of the two
    species: E, J and the displacement form a leapfrog oscillator with
    2 sin(w/2) = w_p, w_p^2 = 2 N_ppc |q| (App. A with <gamma> = 1)."""
    import synth
    ppc, nx, c, Rp = 8, 16, 0.45, 10.0
    qabs = synth.charge_from_skin_depth(c, Rp, ppc, 1.0)
    wp = c / Rp
    assert abs(2 * ppc * qabs - wp * wp) < 1e-15
    x = synth.quiet_positions(np.random.default_rng(1), 1, (nx, 1, 1), ppc)
    u0 = 1e-5
    ue = np.zeros((3, x.shape[1]))
    ue[0] = u0
    up = np.zeros((3, x.shape[1]))
    up[0] = -u0
    P = synth.Plasma(D=1, n=(nx, 1, 1), c=c, E=np.zeros((3, nx)), B=np.zeros((3, nx)),
                     species=[synth.Species(-qabs, -1.0, qabs, x.copy(), ue),
                              synth.Species(qabs, 1.0, qabs, x.copy(), up)])
    st = orc.State(P)
    ex = []
    for _ in range(600):
        st.step()
        ex.append(st.E[0].mean())
    ex = np.array(ex)
    # the k=0 mode is a discrete harmonic oscillator: E^{n+1}+E^{n-1} = 2 cos(w) E^n
    cosw = np.median((ex[2:] + ex[:-2]) / (2 * ex[1:-1]))
    w = math.acos(cosw)
    assert abs(2 * math.sin(w / 2) - wp) < 1e-3 * wp


# ----------------------------------------- 2D out-of-plane current, wrap

def _path_average_jz(x1, x2, dz, q, n):
    """Out-of-plane current of a 2D move, built independently of the
    oracle: along each straight piece of the ZigZag path the current density
    q vz times the first-order (cloud-in-cell) shape, averaged over the
    piece by 3-point Gauss-Legendre quadrature (exact for the quadratic
    product of two linear weights).  The two pieces (x1 -> relay point ->
    x2) each carry half of the out-of-plane displacement (relay at the
    midpoint along non-grid dimensions)."""
    gl_t, gl_w = np.polynomial.legendre.leggauss(3)
    gl_t = 0.5 * (gl_t + 1.0)
    gl_w = 0.5 * gl_w
    J = np.zeros((n[1], n[0]))
    i1, i2 = np.floor(x1), np.floor(x2)
    xr = np.minimum(np.minimum(i1, i2) + 1, np.maximum(np.maximum(i1, i2), 0.5 * (x1 + x2)))
    for a, b, cell in ((x1, xr, i1), (xr, x2, i2)):
        for t, w in zip(gl_t, gl_w):
            p = a + t * (b - a)
            f = p - cell                      # position inside the piece's cell
            for ca in (0, 1):
                for cb in (0, 1):
                    s = (f[0] if ca else 1 - f[0]) * (f[1] if cb else 1 - f[1])
                    J[int(cell[1] + cb) % n[1], int(cell[0] + ca) % n[0]] += q * 0.5 * dz * w * s
    return J.reshape(-1)


def test_2d_out_of_plane_current_is_the_path_average(orc):
    """In 2D3V the out-of-plane current of each ZigZag piece is the path
    average of the particle shape along the piece (Esirkepov 2001's 2D3V
    out-of-plane current, the same path average that continuity forces on
    every component in 3D): midpoint weights plus sigma_a sigma_b dx dy / 12.
    Checked against an independent quadrature of the shape along the path,
    for in-cell moves with dx, dy, dz all nonzero and for moves that cross
    one or two faces; a dropped or sign-flipped dx dy / 12 term misses by
    q dz dx dy / 12."""
    n = (6, 5, 1)
    q = 0.8
    rng = np.random.default_rng(7)
    cases = [((2.2, 1.3), (0.55, 0.6), 0.7),        # in-cell, large in-plane motion
             ((3.9, 2.1), (-0.7, 0.8), -0.4)]       # in-cell, opposite signs
    for _ in range(200):
        x1 = rng.uniform(1.0, 4.0, 2)
        d = rng.uniform(-0.95, 0.95, 2)
        cases.append((tuple(x1), tuple(d), float(rng.uniform(-0.9, 0.9))))
    worst, crossings = 0.0, 0
    for x1, d, dz in cases:
        x1 = np.array(x1)
        x2 = x1 + np.array(d)
        crossings += bool((np.floor(x1) != np.floor(x2)).any())
        J = np.zeros((3, n[0] * n[1]))
        orc.zigzag(2, n, q, x1[:, None], x2[:, None], np.array([d[0], d[1], dz])[:, None], J)
        want = _path_average_jz(x1, x2, dz, q, n)
        worst = max(worst, np.abs(J[2] - want).max())
    assert crossings > 50
    assert worst < 1e-15, worst
    # the term is visible: the first case's cross term q dz dx dy / 12
    assert abs(q * 0.7 * 0.55 * 0.6 / 12) > 1e-2


def test_wrap_edges(orc):
    """C-13: after the periodic wrap every coordinate lies in [0, N), also
    at the edges: a tiny negative value whose sum with N rounds to N becomes
    0, x = N becomes 0, N minus one ulp stays, 2N minus one ulp maps to N
    minus that ulp (exact), and -ulp(N) maps to N - ulp(N)."""
    N = 64
    n = (N, 1, 1)
    ulp_n = np.spacing(float(N))
    x = np.array([[-1e-17, -ulp_n / 4, N - ulp_n, float(N), 2 * N - 2 * ulp_n, -ulp_n, 0.0, 3.5]])
    want = [0.0, 0.0, N - ulp_n, 0.0, N - 2 * ulp_n, N - ulp_n, 0.0, 3.5]
    orc.wrap(1, n, x)
    assert x[0].tolist() == want
    assert (x >= 0).all() and (x < N).all()
    # per dimension in 2D and 3D as well
    x3 = np.array([[-1e-17, 5.0], [float(N), -1e-300], [7.25, 2 * N - 2 * ulp_n]])
    orc.wrap(3, (N, N, N), x3)
    assert x3.tolist() == [[0.0, 5.0], [0.0, 0.0], [7.25, N - 2 * ulp_n]]
