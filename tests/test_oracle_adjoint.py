"""Pins of the oracle's hand-written adjoint (reverse mode) of the step.

Differentiation is an addition to the method (the paper integrates forward
only); the adjoint must be the exact vector-Jacobian product of the forward
step, so it is pinned against central finite differences of the forward
oracle in random directions of the whole state (1D/2D/3D), against the
exact transpose identity for the linear field solver, and against finite
differences of the loss with respect to the workload parameters (shear
amplitude and guide field) that the gradient of config 5 targets.
"""
import math

import numpy as np
import pytest

import oracle
import synth


def perturbed_loss(st, dirs, eps, nsteps):
    s2 = st.copy()
    dx, du, dE, dB = dirs
    for i in range(len(s2.x)):
        s2.x[i] += eps * dx[i]
        oracle.wrap(s2.D, s2.n, s2.x[i])
        s2.u[i] += eps * du[i]
    s2.E += eps * dE
    s2.B += eps * dB
    s2.step(nsteps)
    return oracle.loss_e2(s2)


def small_state(D, seed):
    if D == 2:
        return oracle.State(synth.shear(n=16, ppc=2, seed=seed))
    n = (24, 1, 1) if D == 1 else (6, 6, 6)
    p = synth.small_random(D, n, 4 if D == 1 else 1, theta=0.2, field_amp=0.02, seed=seed, q=2e-3)
    return oracle.State(p)


@pytest.mark.parametrize("D", [1, 2, 3])
def test_adjoint_matches_directional_finite_differences(D):
    """<grad L, delta> equals (L(s + h delta) - L(s - h delta)) / 2h for
    random directions delta of (x, u, E, B), h = 1e-6, over 4 steps."""
    st = small_state(D, 10 + D)
    nsteps = 4
    L, lx, lu, lE, lB = oracle.adjoint_run(st, nsteps)
    rng = np.random.default_rng(D)
    for trial in range(3):
        dirs = ([0.2 * rng.standard_normal(x.shape) for x in st.x],
                [rng.standard_normal(u.shape) for u in st.u],
                1e-3 * rng.standard_normal(st.E.shape), 1e-3 * rng.standard_normal(st.B.shape))
        ad = sum(float((a * b).sum()) for a, b in zip(lx, dirs[0])) + \
            sum(float((a * b).sum()) for a, b in zip(lu, dirs[1])) + \
            float((lE * dirs[2]).sum()) + float((lB * dirs[3]).sum())
        h = 1e-6
        fd = (perturbed_loss(st, dirs, h, nsteps) - perturbed_loss(st, dirs, -h, nsteps)) / (2 * h)
        assert abs(fd - ad) <= 1e-6 * abs(ad), (trial, fd, ad)


def test_field_adjoint_is_exact_transpose():
    """Without particles the step is linear in (E, B): <lambda, M delta> =
    <M^T lambda, delta> to round-off (M delta evaluated exactly by linearity)."""
    p = synth.small_random(3, (6, 5, 4), 1, seed=2)
    for sp in p.species:
        sp.x = sp.x[:, :0].copy()
        sp.u = sp.u[:, :0].copy()
    st = oracle.State(p)
    rng = np.random.default_rng(3)
    lE0, lB0 = rng.standard_normal(st.E.shape), rng.standard_normal(st.B.shape)
    dE, dB = rng.standard_normal(st.E.shape), rng.standard_normal(st.B.shape)
    s2 = st.copy()
    s2.E[:] = dE
    s2.B[:] = dB
    s2.step(3)
    lhs = float((lE0 * s2.E).sum() + (lB0 * s2.B).sum())
    lE, lB = lE0.copy(), lB0.copy()
    st3 = st.copy()
    for _ in range(3):
        st3.step_adjoint([], [], lE, lB)
    rhs = float((lE * dE).sum() + (lB * dB).sum())
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_parameter_gradients_match_finite_differences():
    """dL/dA (shear amplitude, u += A sin(2 pi y / n) x) and dL/dB0 (uniform
    guide field) from the adjoint of the initial state agree with central
    differences of the full pipeline (generator + 6 steps) to 1e-6."""
    n, ppc, A, nsteps = 16, 2, 0.1, 6
    base = synth.shear(n=n, ppc=ppc, amp=A, seed=7)
    B0 = base.meta["B0"]
    st = oracle.State(base)
    L, lx, lu, lE, lB = oracle.adjoint_run(st, nsteps)
    dLdA = sum(float((lu[i][0] * np.sin(2 * math.pi * st.x[i][1] / n)).sum()) for i in range(2))
    dLdB0 = float(lB[2].sum())

    def loss(amp, b0):
        s = oracle.State(synth.shear(n=n, ppc=ppc, amp=amp, seed=7, B0=b0))
        s.step(nsteps)
        return oracle.loss_e2(s)
    h = 1e-6
    fdA = (loss(A + h, B0) - loss(A - h, B0)) / (2 * h)
    fdB = (loss(A, B0 + h) - loss(A, B0 - h)) / (2 * h)
    assert abs(fdA - dLdA) < 1e-6 * abs(dLdA), (fdA, dLdA)
    assert abs(fdB - dLdB0) < 1e-6 * abs(dLdB0), (fdB, dLdB0)


def test_zigzag_transverse_current_jumps_at_face_crossing():
    """App. D relay point: min(min(i1,i2)+1, max(max(i1,i2), midpoint)) is
    the midpoint while both ends share a cell and the face once x2 crosses
    it, so the transverse current jumps there (the loss is only piecewise
    smooth) while the charge flux through every face stays continuous."""
    n, D = (4, 4, 1), 2
    J = []
    for x2x in (1 - 1e-9, 1 + 1e-9):
        x1 = np.array([[0.7], [0.5]])
        x2 = np.array([[x2x], [0.7]])
        disp = np.array([[x2x - 0.7], [0.2], [0.1]])
        j = np.zeros((3, 16))
        oracle.zigzag(D, n, 1.0, x1, x2, disp, j)
        J.append(j)
    # net flux through every x face line and y face line, and the total of
    # each component: continuous
    fx = [j[0].reshape(4, 4).sum(axis=0) for j in J]
    fy = [j[1].reshape(4, 4).sum(axis=1) for j in J]
    assert np.abs(fx[0] - fx[1]).max() < 1e-8 and np.abs(fy[0] - fy[1]).max() < 1e-8
    assert abs(J[0][2].sum() - J[1][2].sum()) < 1e-8
    # J_y at node (0, 0): midpoint relay gives q dy (1 - (x1+x2)/2) = 0.03,
    # face relay gives q (dy/2)(1 - (x1+1)/2) = 0.015
    assert abs(J[0][1][0] - 0.03) < 1e-8 and abs(J[1][1][0] - 0.015) < 1e-8


def test_parameter_gradient_against_fd_sweep():
    """With more particles and steps some finite-difference intervals hold a
    face crossing (see above) and miss by jump/2h.  Such an interval shows
    itself by forward and backward one-sided differences that disagree; the
    central differences of the other intervals agree with the adjoint."""
    n, ppc, A, nsteps = 32, 8, 0.1, 12
    B0 = 0.078772
    st = oracle.State(synth.shear(n=n, ppc=ppc, amp=A, B0=B0))
    L, lx, lu, lE, lB = oracle.adjoint_run(st, nsteps)
    dLdA = sum(float((lu[i][0] * np.sin(2 * math.pi * st.x[i][1] / n)).sum()) for i in range(2))
    dLdB0 = float(lB[2].sum())

    def loss(amp, b0):
        s = oracle.State(synth.shear(n=n, ppc=ppc, amp=amp, B0=b0))
        s.step(nsteps)
        return oracle.loss_e2(s)
    L0 = loss(A, B0)
    clean = {"A": 0, "B0": 0}
    for h in (1e-7, 1e-8, 1e-9):
        for key, g, (lp, lm) in (("A", dLdA, (loss(A + h, B0), loss(A - h, B0))),
                                 ("B0", dLdB0, (loss(A, B0 + h), loss(A, B0 - h)))):
            fwd, bwd, cen = (lp - L0) / h, (L0 - lm) / h, (lp - lm) / (2 * h)
            if abs(fwd - bwd) <= 1e-5 * abs(cen):
                clean[key] += 1
                assert abs(cen - g) < 1e-6 * abs(g), (key, h, cen, g)
    assert clean["A"] >= 1 and clean["B0"] >= 1
