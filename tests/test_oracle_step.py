"""Pins of the oracle's full step and of the synthetic inputs.

* P-9: Gauss's law and div B are preserved to round-off by the full step
  (App. B: Yee staggering plus a charge-conserving deposit).
* P-11: the Maxwell-Juttner sampler's mean Lorentz factor matches
  K1(1/theta)/K2(1/theta) + 3 theta and the paper's printed value; the
  turbulence forcing has the discrete energy its mode sum fixes and zero
  discrete divergence.
* Golden values printed in the paper (tests/golden/paper_values.txt).
"""
import math
import os

import numpy as np
import pytest

import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_values.txt")


def golden():
    out = {}
    for line in open(GOLD):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        name, val, tol, cite = [s.strip() for s in line.split("|")]
        out[name] = (float(val), float(tol), cite)
    return out


def test_weibel_full_run_preserves_gauss_and_divb(orc):
    """P-9 on the 1D3V Weibel workload: 200 FP64 steps."""
    p = synth.weibel()
    st = orc.State(p)
    g0 = st.gauss_residual()
    assert np.abs(g0).max() < 1e-15          # co-located pairs: rho = 0, E = 0
    st.step(200)
    assert np.abs(st.gauss_residual()).max() < 1e-12
    assert np.abs(st.div_b()).max() < 1e-12
    # the beams have done something: field energy grew from zero
    uf, uk = st.energies()
    assert uf > 0 and uk > 0


@pytest.mark.parametrize("D", [2, 3])
def test_multi_d_full_run_preserves_gauss_and_divb(orc, D):
    """P-9 in 2D (turbulence-shaped, forcing on) and 3D (thermal)."""
    if D == 2:
        p = synth.turbulence(n=48, ppc=4, seed=5)
    else:
        rng = np.random.default_rng(3)
        n = (8, 8, 8)
        x = synth.quiet_positions(rng, 3, n, 3)
        q = 2e-3
        P = [synth.Species(-q, -1.0, q, x.copy(), synth.sample_mj(rng, 0.3, x.shape[1])),
             synth.Species(q, 1.0, q, x.copy(), synth.sample_mj(rng, 0.3, x.shape[1]))]
        B = np.zeros((3, 512))
        B[2] = 0.1
        p = synth.Plasma(D=3, n=n, c=0.45, species=P, E=np.zeros((3, 512)), B=B)
    st = orc.State(p)
    assert np.abs(st.gauss_residual()).max() < 1e-15
    assert np.abs(st.div_b()).max() < 1e-12
    st.step(30)
    assert np.abs(st.gauss_residual()).max() < 1e-12
    assert np.abs(st.div_b()).max() < 1e-12


def test_gauss_pin_catches_a_sign_error(orc):
    """Negative control for P-9: depositing the current with the wrong sign
    (E += J instead of E -= J) breaks Gauss's law at first order."""
    p = synth.turbulence(n=32, ppc=2, seed=6)
    st = orc.State(p)
    st.step(1)
    g_ok = np.abs(st.gauss_residual()).max()
    # redo with the sign flipped: E_bad = E + 2 J reproduces E += J
    st.E += 2.0 * st.J
    g_bad = np.abs(st.gauss_residual()).max()
    assert g_ok < 1e-14 and g_bad > 1e-6


@pytest.mark.parametrize("theta", [0.01, 0.1, 0.3, 1.0])
def test_mj_sampler_mean_gamma(theta):
    """P-11: sample mean of gamma within 4 standard errors of the exact
    K1(1/theta)/K2(1/theta) + 3 theta (Bessel values from scipy)."""
    rng = np.random.default_rng(17)
    u = synth.sample_mj(rng, theta, 400000)
    g = np.sqrt(1 + (u * u).sum(0))
    want = synth.mean_gamma_mj(theta)
    se = g.std() / math.sqrt(g.size)
    assert abs(g.mean() - want) < 4 * se
    # isotropy: mean of each component is 0, equal second moments
    m2 = (u * u).mean(1)
    assert np.abs(u.mean(1)).max() < 5 * math.sqrt(m2.max() / u.shape[1])
    assert np.ptp(m2) < 0.02 * m2.mean()


def test_mj_mean_gamma_matches_paper_value():
    """The paper prints <gamma> about 1.6 at theta = 0.3."""
    val, tol, _ = golden()["mean_gamma_theta_0.3"]
    assert abs(synth.mean_gamma_mj(0.3) - val) < tol
    # non-relativistic expansion 1 + 3/2 theta + 15/8 theta^2 + O(theta^3)
    th = 1e-4
    assert abs(synth.mean_gamma_mj(th) - (1 + 1.5 * th + 15 / 8 * th * th)) < 1e-11


def test_boost_flux_weighting():
    """A cold population (theta -> 0) boosted to gamma_b gets u_x = sqrt(gamma_b^2-1)."""
    rng = np.random.default_rng(2)
    u = synth.boost_x(rng, np.zeros((3, 10)), 3.0, -1.0)
    assert np.allclose(u[0], -math.sqrt(8.0), rtol=0, atol=1e-14)


def test_turbulence_forcing_energy_and_divergence(orc):
    """P-11: the discrete forcing has box-averaged |dB_perp|^2 equal to the
    mode sum of beta^2/4 ((L/pi) sin(k/2))^2 over both components (exact by
    orthogonality on the lattice), within 3e-3 of the paper's continuum dB^2
    for N = 8 on a 256 box (the lattice factor (sin(k/2)/(k/2))^2), and zero discrete divergence."""
    n = (256, 256, 1)
    dB = 0.7
    rng = np.random.default_rng(4)
    Bxy = synth.turbulence_field(rng, n, dB, nmodes=8)
    L = 256.0
    pred = 0.0
    for m in range(1, 9):
        for k in range(1, 9):
            beta = 2 * dB / (8 * math.sqrt(m * m + k * k))
            fx = (L / math.pi) * math.sin(math.pi * k / L)
            fy = (L / math.pi) * math.sin(math.pi * m / L)
            pred += beta * beta / 4 * (fx * fx + fy * fy)
    got = (Bxy ** 2).sum(0).mean()
    assert abs(got - pred) < 1e-12 * pred
    assert abs(got - dB * dB) < 3e-3 * dB * dB
    B = np.zeros((3, 256 * 256))
    B[:2] = Bxy
    assert np.abs(orc.div_face(n, B)).max() < 1e-13
    val, _, _ = golden()["forcing_modes_N"]
    assert val == 8


def test_unit_system_constants():
    """App. A: |q| from the skin depth and B0 from sigma, on the turbulence
    workload (R_p = 3, 16 ppc/species, theta = 0.3, sigma = 10)."""
    mg = synth.mean_gamma_mj(0.3)
    q = synth.charge_from_skin_depth(0.45, 3.0, 16, mg)
    B0 = synth.b0_from_sigma(10.0, 0.45, 16, q, mg)
    # sigma = B0^2 / (N_ppc m c^2 <gamma> (1+m-/m+)) recovered
    assert abs(B0 ** 2 / (16 * q * 0.45 ** 2 * mg * 2) - 10.0) < 1e-12
    # w_p^2 = |q| N_ppc (1+m-/m+) / <gamma> recovered
    assert abs(q * 16 * 2 / mg - (0.45 / 3.0) ** 2) < 1e-15
    # for pairs B0 = sqrt(sigma) c^2 <gamma> / R_p
    assert abs(B0 - math.sqrt(10.0) * 0.45 ** 2 * mg / 3.0) < 1e-14


def test_paper_printed_physics_numbers():
    """Printed numbers used to shape the inputs: the filamentation growth
    rate at gamma_b = 3 and the MHD jump conditions at Gamma = 10."""
    g = golden()
    gb = 3.0
    beta = math.sqrt(1 - 1 / gb ** 2)
    val, tol, _ = g["weibel_growth_gamma_3"]
    assert abs(beta * math.sqrt(2 / gb) - val) < tol
    Gam, gad = 10.0, 4.0 / 3.0
    comp = 1 + (Gam + 1) / (Gam * (gad - 1))
    bsh = (gad - 1) * (Gam - 1) / Gam
    val, tol, _ = g["shock_compression_mhd"]
    assert abs(comp - val) < tol
    val, tol, _ = g["shock_speed_mhd"]
    assert abs(bsh - val) < tol


@pytest.mark.parametrize("D,nthreads", [(1, 3), (2, 4), (3, 5)])
def test_threaded_step_matches_single_thread(D, nthreads):
    """The all-thread CPU baseline computes the single-thread oracle's step:
    particles bit for bit, J and E to the rounding of the reordered current
    sums (relative 1e-14), over 3 steps."""
    import oracle
    n = {1: (64,), 2: (32, 24), 3: (12, 12, 8)}[D]
    plasma = synth.small_random(D, n, 6, seed=70 + D, field_amp=0.05)
    a = oracle.State(plasma)
    b = oracle.State(plasma)
    a.step(3)
    b.step(3, threads=nthreads)
    for s in range(2):
        assert np.abs(a.x[s] - b.x[s]).max() < 1e-12 and np.abs(a.u[s] - b.u[s]).max() < 1e-13
    for x, y in ((a.J, b.J), (a.E, b.E), (a.B, b.B)):
        assert np.linalg.norm(x - y) <= 1e-14 * np.linalg.norm(x)
    # one step from the same state: particles identical bit for bit
    c, d = oracle.State(plasma), oracle.State(plasma)
    c.step(1)
    d.step(1, threads=nthreads)
    for s in range(2):
        assert np.array_equal(c.x[s], d.x[s]) and np.array_equal(c.u[s], d.u[s])


@pytest.mark.parametrize("D", [1, 2, 3])
def test_split_step_equals_step(D):
    """push_particles + finish_step run the routines of orc_step in its
    order: bit for bit the same state."""
    import oracle
    n = {1: (40,), 2: (24, 16), 3: (8, 8, 8)}[D]
    plasma = synth.small_random(D, n, 4, seed=80 + D, field_amp=0.05)
    a, b = oracle.State(plasma), oracle.State(plasma)
    for _ in range(2):
        a.step(1)
        b.finish_step(b.push_particles())
    for s in range(2):
        assert np.array_equal(a.x[s], b.x[s]) and np.array_equal(a.u[s], b.u[s])
    for x, y in ((a.E, b.E), (a.B, b.B), (a.J, b.J)):
        assert np.array_equal(x, y)
