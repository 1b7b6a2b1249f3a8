"""Brute-force single-particle pin of the oracle's particle recurrence.

The relativistic Boris update of App. C is a half electric kick, a pure
rotation of the four-velocity about the magnetic field, and a second half
kick; the rotation angle is 2 arctan |t| with t = s B / (2 c gamma_1).  Here
that update is written a second way, as an explicit rotation (Rodrigues'
formula with the angle computed by arctan) instead of the oracle's
cross-product form, and evaluated with 50 significant digits (mpmath), then
followed by the position advance of Eq. (fdX).  Over 500 steps in a uniform
magnetic field and in crossed fields:

* local error: from every one of the 500 high-precision states, one
  double-precision step of the oracle lands within 8 units of double
  rounding (relative to |u| and |x|) of the high-precision step;
* global error: the oracle's own 500-step orbit stays within the sum of
  those local errors, 500 x 8 units of double rounding, of the
  high-precision orbit (the rotation keeps |u|, so u errors add up without
  growing; x adds the displacements).

A dropped term, a wrong sign or a swapped operand in either form moves a
single step at first order in the fields, many orders of magnitude beyond
these bounds.
"""
import numpy as np
import pytest

mp = pytest.importorskip("mpmath")
DIGITS = 50
STEPS = 500


def mp_step(u, x, E, B, c, s):
    """One step in mpmath: half kick, rotation about t by -2 arctan|t|
    (Rodrigues), half kick, then x += c u / gamma(u)."""
    c = mp.mpf(c)
    s = mp.mpf(s)
    um = [c * u[i] + s * E[i] / 2 for i in range(3)]
    g1 = mp.sqrt(1 + (um[0] ** 2 + um[1] ** 2 + um[2] ** 2) / c ** 2)
    t = [s * B[i] / (2 * c * g1) for i in range(3)]
    tn = mp.sqrt(t[0] ** 2 + t[1] ** 2 + t[2] ** 2)
    if tn == 0:
        up = um
    else:
        k = [ti / tn for ti in t]
        th = -2 * mp.atan(tn)
        kxu = [k[1] * um[2] - k[2] * um[1], k[2] * um[0] - k[0] * um[2], k[0] * um[1] - k[1] * um[0]]
        kdu = k[0] * um[0] + k[1] * um[1] + k[2] * um[2]
        ct, st = mp.cos(th), mp.sin(th)
        up = [um[i] * ct + kxu[i] * st + k[i] * kdu * (1 - ct) for i in range(3)]
    un = [(up[i] + s * E[i] / 2) / c for i in range(3)]
    g = mp.sqrt(1 + un[0] ** 2 + un[1] ** 2 + un[2] ** 2)
    xn = [x[i] + c * un[i] / g for i in range(3)]
    return un, xn


CASES = {
    # uniform B, relativistic gyration (gamma ~ 2.3)
    "uniform_b": dict(c=0.45, s=-1.0, E=(0.0, 0.0, 0.0), B=(0.03, -0.02, 0.31), u0=(1.7, -0.9, 0.6)),
    # crossed fields, |E| < |B|: drifting gyration
    "crossed": dict(c=0.45, s=1.0, E=(0.0, 0.012, 0.0), B=(0.0, 0.0, 0.2), u0=(0.4, 0.1, -0.3)),
    # crossed fields with a parallel E component: acceleration along B
    "crossed_parallel": dict(c=0.3, s=-1.0, E=(0.004, 0.01, 0.002), B=(0.05, 0.0, 0.15), u0=(-0.2, 0.6, 0.05)),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_oracle_recurrence_against_50_digit_rotation_form(orc, name):
    cs = CASES[name]
    eps = np.finfo(float).eps
    with mp.workdps(DIGITS):
        E = [mp.mpf(v) for v in cs["E"]]
        B = [mp.mpf(v) for v in cs["B"]]
        u = [mp.mpf(v) for v in cs["u0"]]
        x = [mp.mpf(0)] * 3
        states = []
        for _ in range(STEPS):
            states.append((u, x))
            u, x = mp_step(u, x, E, B, cs["c"], cs["s"])
        states.append((u, x))
        ref_u = np.array([[float(v) for v in st[0]] for st in states])
        ref_x = np.array([[float(v) for v in st[1]] for st in states])
    Ep = np.array(cs["E"], float).reshape(3, 1)
    Bp = np.array(cs["B"], float).reshape(3, 1)
    # local error: one oracle step from each high-precision state (all 500
    # states as 500 particles of one call)
    u0 = np.ascontiguousarray(ref_u[:-1].T)
    x0 = np.ascontiguousarray(ref_x[:-1].T)
    ones = np.ones((1, STEPS))
    orc.boris(cs["c"], cs["s"], Ep * ones, Bp * ones, u0)
    orc.move(3, cs["c"], u0, x0)
    du = np.abs(u0.T - ref_u[1:]).max(axis=1) / np.abs(ref_u[1:]).max(axis=1)
    dx = np.abs(x0.T - ref_x[1:]).max(axis=1) / np.abs(ref_x[1:]).max(axis=1)
    # global error: the oracle's own orbit
    ud = np.array(cs["u0"], float).reshape(3, 1).copy()
    xd = np.zeros((3, 1))
    got_u, got_x = [ud[:, 0].copy()], [xd[:, 0].copy()]
    for _ in range(STEPS):
        orc.boris(cs["c"], cs["s"], Ep, Bp, ud)
        orc.move(3, cs["c"], ud, xd)
        got_u.append(ud[:, 0].copy())
        got_x.append(xd[:, 0].copy())
    eu = np.abs(np.array(got_u) - ref_u).max() / np.abs(ref_u).max()
    ex = np.abs(np.array(got_x) - ref_x).max() / np.abs(ref_x).max()
    print(f"{name}: local u {du.max() / eps:.1f} eps, x {dx.max() / eps:.1f} eps; "
          f"global after {STEPS} steps u {eu:.2e}, x {ex:.2e}")
    assert du.max() < 8 * eps and dx.max() < 8 * eps, (du.max() / eps, dx.max() / eps)
    assert eu < STEPS * 8 * eps and ex < STEPS * 8 * eps, (eu, ex)


def test_rotation_form_detects_a_dropped_term(orc):
    """The comparison is sharp: dropping the second half kick from the
    high-precision form moves u by s E / (2 c) after one step."""
    cs = CASES["crossed"]
    with mp.workdps(DIGITS):
        E = [mp.mpf(v) for v in cs["E"]]
        B = [mp.mpf(v) for v in cs["B"]]
        u = [mp.mpf(v) for v in cs["u0"]]
        un, _ = mp_step(u, [mp.mpf(0)] * 3, E, B, cs["c"], cs["s"])
        bad = [float(un[i] - mp.mpf(cs["s"]) * E[i] / (2 * mp.mpf(cs["c"]))) for i in range(3)]
    ud = np.array(cs["u0"], float).reshape(3, 1).copy()
    orc.boris(cs["c"], cs["s"], np.array(cs["E"], float).reshape(3, 1), np.array(cs["B"], float).reshape(3, 1), ud)
    assert np.abs(ud[:, 0] - np.array(bad)).max() > 1e-3
