"""Pins of the oracle's energy diagnostics (field energy 1/2 sum(E^2 + B^2)
and kinetic energy sum m c^2 (gamma - 1), the reading the energy report
takes; the paper states no energy diagnostic) against closed forms that do
not restate the formulas:

* a single discrete lattice mode sin(2 pi m i / n) has sum of squares n/2
  exactly (orthogonality on the lattice), so the field energy of a few
  modes in different components is a known number;
* momenta with integer Lorentz factors (|u|^2 = 3, 8, 15) give kinetic
  energies of 1, 2, 3 m c^2;
* a Maxwell-Juttner population has mean kinetic energy
  m c^2 (K1(1/theta)/K2(1/theta) + 3 theta - 1), from the Bessel functions.

A dropped factor 1/2, a missing component, gamma in place of gamma - 1 or
a wrong power of c fails one of them."""
import math

import numpy as np
import pytest

import oracle
import synth


@pytest.mark.parametrize("D,n", [(1, (64, 1, 1)), (2, (32, 24, 1)), (3, (12, 10, 8))])
def test_field_energy_of_lattice_modes(D, n):
    N = n[0] * n[1] * n[2]
    c = np.arange(N)
    idx = [c % n[0], (c // n[0]) % n[1], c // (n[0] * n[1])]
    E = np.zeros((3, N))
    B = np.zeros((3, N))
    # one mode per component along different axes and wave numbers; every
    # mode is a sine or cosine of 2 pi m i / n with 0 < m < n/2, whose
    # squares sum to N/2 over the box
    amps = [0.3, -1.7, 0.9, 2.5, -0.4, 1.1]
    for comp in range(6):
        ax = comp % D
        m = 1 + comp % 3
        arg = 2 * math.pi * m * idx[ax] / n[ax]
        v = amps[comp] * (np.sin(arg) if comp % 2 == 0 else np.cos(arg))
        (E if comp < 3 else B)[comp % 3] = v
    expect = 0.5 * sum(a * a for a in amps) * N / 2
    got = oracle.field_energy(n, E, B)
    assert abs(got - expect) < 1e-12 * expect


def test_kinetic_energy_integer_gammas():
    mass, c = 0.37, 0.45
    # |u|^2 = 3, 8, 15 -> gamma = 2, 3, 4; directions mixed
    u = np.array([[math.sqrt(3.0), 0.0, 1.0, 2.0, 0.0],
                  [0.0, math.sqrt(8.0), 1.0, 2.0, 0.0],
                  [0.0, 0.0, 1.0, math.sqrt(7.0), 0.0]])
    # gammas 2, 3, 2, 4, 1: kinetic energies 1, 2, 1, 3, 0 m c^2
    got = oracle.kinetic_energy(mass, c, u)
    assert abs(got - 7.0 * mass * c * c) < 1e-14
    assert oracle.kinetic_energy(mass, c, np.zeros((3, 4))) == 0.0


@pytest.mark.parametrize("theta", [0.3, 3.0])
def test_kinetic_energy_of_maxwell_juttner_population(theta):
    """Mean over 400,000 samples within 5 standard errors of the closed form."""
    rng = np.random.default_rng(11)
    n = 400_000
    u = synth.sample_mj(rng, theta, n)
    mass, c = 1.3, 0.45
    got = oracle.kinetic_energy(mass, c, u) / n
    from scipy import special as sp
    x = 1.0 / theta
    expect = mass * c * c * (sp.kve(1, x) / sp.kve(2, x) + 3.0 * theta - 1.0)
    g = np.sqrt(1.0 + (u * u).sum(0))
    se = mass * c * c * g.std() / math.sqrt(n)
    assert abs(got - expect) < 5 * se, (got, expect, se)


def test_state_energies_sum_over_species():
    """State.energies adds every species' kinetic energy with its own mass."""
    p = synth.small_random(2, (8, 8), 1, seed=5)
    st = oracle.State(p)
    for s in range(2):
        st.u[s][:] = 0.0
    st.u[0][0, :] = math.sqrt(3.0)        # gamma 2 for every particle of species 0
    st.u[1][1, :] = math.sqrt(8.0)        # gamma 3 for species 1
    _, uk = st.energies()
    c = p.c
    expect = (p.species[0].m * st.u[0].shape[1] * 1.0 + p.species[1].m * st.u[1].shape[1] * 2.0) * c * c
    assert abs(uk - expect) < 1e-12 * expect
