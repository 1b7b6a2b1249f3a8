"""Physics pin of the oracle's full step: the filamentation (Weibel)
instability of Sect. 5.1.

Two counter-streaming pair beams with Lorentz factor gamma_b = 3 stream
along y across a 1D grid along x (512 cells, 64 particles per cell per
species, beam-frame temperature 0.01, skin depth 10 cells).  The paper
gives the growth rate delta / w_p = beta_b sqrt(2 / gamma_b) (0.7698 at
gamma_b = 3, tests/golden/paper_values.txt); its w_p normalisation (per
beam or total, with or without the mean Lorentz factor) is open by up to
a factor sqrt 2, so the check is soft: the magnetic energy must grow
exponentially (a straight line in log over the linear phase) at twice a
rate within a factor sqrt 2 of the formula, with w_p = c / R_p of the code
units (App. A).

Control: the same beams streaming along x, the grid direction (the
two-stream geometry), have no filamentation mode on this grid; their
magnetic energy only accumulates the thermal noise of the transverse
currents and ends the same steps more than ten times below.

The pin sees mistakes in the current: the step assembled from the oracle's
own routines, with Jx and Jy exchanged or Jy dropped before add_cur, fails
it (the last test plants both on the CPU).
"""
import math

import numpy as np
import pytest

import synth

STEPS = 101
WINDOW = (40, 100)      # the linear phase of this seed: magnetic energy 3e-5 .. 2e-3


def magnetic_energy_history(plasma, steps, mistake=None):
    """Magnetic energy after each oracle step; with a mistake, the step is
    assembled from the oracle's routines in the order of its step, and the
    current is altered before add_cur."""
    import oracle
    st = oracle.State(plasma)
    D, n, c = st.D, st.n, st.c
    out = []
    for _ in range(steps):
        if mistake is None:
            st.step(1)
        else:
            ends = st.push_particles()
            oracle.advance_b(D, n, 0.5 * c, st.E, st.B)
            oracle.advance_e(D, n, c, st.B, st.E)
            st.J[:] = 0.0
            for s in range(len(st.x)):
                x2 = np.ascontiguousarray(ends[s])
                oracle.zigzag(D, n, st.q[s], st._x1[s], x2, st._disp[s], st.J)
                oracle.wrap(D, n, x2)
                st.x[s] = x2
            if mistake == "exchange_jx_jy":
                st.J[[0, 1]] = st.J[[1, 0]]
            elif mistake == "drop_jy":
                st.J[1] = 0.0
            oracle.add_current(n, st.J, st.E)
        out.append(0.5 * float(np.sum(st.B * st.B)))
    return np.array(out)


def pin_holds(ub, wp, f):
    rate, r2 = growth_rate(ub, WINDOW, wp)
    return r2 > 0.995 and f / math.sqrt(2.0) < rate < f * math.sqrt(2.0) and ub[WINDOW[1]] > 30.0 * ub[WINDOW[0]]


def growth_rate(ub, window, wp):
    """delta / w_p from a straight-line fit of log(magnetic energy), and
    the fit's R^2."""
    a, b = window
    t = np.arange(a, b)
    y = np.log(ub[a:b])
    slope, icpt = np.polyfit(t, y, 1)
    res = y - (slope * t + icpt)
    r2 = 1.0 - np.sum(res * res) / np.sum((y - y.mean()) ** 2)
    return slope / 2.0 / wp, r2


def formula(gamma_b):
    beta = math.sqrt(1.0 - 1.0 / gamma_b ** 2)
    return beta * math.sqrt(2.0 / gamma_b)


def test_oracle_filamentation_growth_rate():
    p = synth.weibel(beam_axis=1)
    wp = p.c / p.meta["Rp"]
    ub = magnetic_energy_history(p, STEPS)
    rate, r2 = growth_rate(ub, WINDOW, wp)
    f = formula(p.meta["gamma_b"])
    print(f"oracle filamentation: delta/w_p = {rate:.4f} (R^2 {r2:.5f}), formula {f:.4f}, ratio {rate / f:.3f}")
    assert r2 > 0.995
    assert f / math.sqrt(2.0) < rate < f * math.sqrt(2.0)
    # grown by orders of magnitude over the window
    assert ub[WINDOW[1]] > 30.0 * ub[WINDOW[0]]


def test_two_stream_geometry_grows_no_magnetic_field():
    p = synth.weibel(beam_axis=0)
    ub = magnetic_energy_history(p, STEPS)
    q = synth.weibel(beam_axis=1)
    uf = magnetic_energy_history(q, STEPS)
    print(f"magnetic energy after {STEPS} steps: beams along x {ub[-1]:.3e}, along y {uf[-1]:.3e}")
    assert ub[-1] < 0.1 * uf[-1]


@pytest.mark.parametrize("mistake", ["exchange_jx_jy", "drop_jy"])
def test_growth_pin_catches_current_mistakes(mistake):
    p = synth.weibel(beam_axis=1)
    wp = p.c / p.meta["Rp"]
    f = formula(p.meta["gamma_b"])
    ub = magnetic_energy_history(p, STEPS, mistake)
    rate, r2 = growth_rate(ub, WINDOW, wp)
    print(f"{mistake}: delta/w_p = {rate:.4f} (R^2 {r2:.4f})")
    assert not pin_holds(ub, wp, f)
