"""GPU reverse mode (adjoint of the fused step) through the C ABI.

* One step, random adjoints of every output: the GPU FP64 adjoint against
  the oracle's hand-written adjoint (which is pinned to finite differences on
  the CPU), relative L2 1e-10 per array.
* Several steps over checkpoint windows, loss sum |E^N|^2: same comparison.
* Gradients of the loss with respect to plasma parameters of a sheared,
  magnetised pair plasma (drift amplitude A, guide field B0) through
  torch.autograd: GPU adjoint (FP64 and FP32) against central finite
  differences of the FP64 forward, 1e-4 relative (1e-6 for FP64).

The ZigZag relay point jumps from the segment midpoint to the cell face
when an end point crosses a face (App. D), so the transverse current and the
loss are only piecewise smooth: a finite difference whose interval holds
such a crossing of any particle is off by (jump)/2h, while the adjoint is
the derivative of the smooth piece.  The finite differences are therefore
taken over a sweep of h; estimates free of crossings agree with each other,
and the adjoint must agree with at least two of the three.
"""
import math

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def make_sim(plasma, T, prec):
    from paper_1906_06306_amd import _lib as L
    from paper_1906_06306_amd.sim import PicSim
    print(f"[gpu] tracked PicSim D={plasma.D} n={plasma.n} T={T} prec={prec} np={plasma.nparticles}", flush=True)
    return PicSim(plasma, tile=T, precision=prec, capacity_factor=2.0, options=L.PIC_OPT_TRACK)


CASES = [
    (1, (64, 1, 1), (16, 1, 1), 16),
    (2, (32, 24, 1), (8, 8, 1), 6),
    (3, (16, 8, 8), (8, 4, 4), 2),
]


def slot_to_input(sim, ids_now, ids_init):
    """For every occupied slot of the current state (one step after init):
    the input index of its particle."""
    _, _, _, off, cnt = sim.particle_views()
    off, cnt = off.cpu().numpy(), cnt.cpu().numpy()
    slots = np.concatenate([np.arange(o, o + c) for o, c in zip(off.ravel(), cnt.ravel())])
    return slots, ids_init[ids_now[slots]]


@pytest.mark.parametrize("D,n,T,ppc", CASES)
def test_adjoint_one_step_matches_oracle(D, n, T, ppc):
    """Random adjoints of x^{n+1}, u^{n+1/2}, E^{n+1}, B^{n+1/2}, strong
    charge (the deposit adjoint matters): FP64 GPU vs oracle."""
    from paper_1906_06306_amd import adjoint
    plasma = synth.small_random(D, n, ppc, seed=41 + D, field_amp=0.05, q=0.05)
    sim = make_sim(plasma, T, "fp64")
    ids0 = sim.ids_host()
    ck = adjoint.forward(sim, 1)
    ids1 = sim.ids_host()
    assert sim.error() == 0
    rng = np.random.default_rng(7 + D)
    npart = [sp.x.shape[1] for sp in plasma.species]
    lx = [rng.standard_normal((D, k)) for k in npart]
    lu = [rng.standard_normal((3, k)) for k in npart]
    N = int(np.prod(n))
    lE = rng.standard_normal((3, N))
    lB = rng.standard_normal((3, N))
    # GPU: adjoints placed at the particles' slots after the step
    slots, inp = slot_to_input(sim, ids1, ids0)
    lx_all, lu_all = np.concatenate(lx, axis=1), np.concatenate(lu, axis=1)
    assert np.array_equal(np.sort(inp), np.arange(sum(npart)))
    la, ua, _, _ = sim.adjoint_buffers()
    dev = sim.device
    la[:, torch.as_tensor(slots, device=dev)] = torch.as_tensor(lx_all[:, inp], device=dev)
    ua[:, torch.as_tensor(slots, device=dev)] = torch.as_tensor(lu_all[:, inp], device=dev)
    gl = adjoint.backward(sim, ck, 1, torch.as_tensor(lE, device=dev), torch.as_tensor(lB, device=dev),
                          lpos=la, lu=ua)
    g_lx, g_lu, g_lE, g_lB = (t.cpu().numpy() for t in gl)
    assert sim.error() == 0
    # oracle, from the input state (input order)
    st = oracle.State(plasma)
    o_lx = [a.copy() for a in lx]
    o_lu = [a.copy() for a in lu]
    o_lE, o_lB = lE.copy(), lB.copy()
    st.step_adjoint(o_lx, o_lu, o_lE, o_lB)
    tol = 1e-10
    assert rel(g_lE, o_lE) < tol, rel(g_lE, o_lE)
    assert rel(g_lB, o_lB) < tol, rel(g_lB, o_lB)
    sl = sim.input_slices()
    for s in range(2):
        a = sl[(0, s)]
        assert rel(g_lx[:, a], o_lx[s]) < tol, (s, rel(g_lx[:, a], o_lx[s]))
        assert rel(g_lu[:, a], o_lu[s]) < tol, (s, rel(g_lu[:, a], o_lu[s]))
    sim.close()


@pytest.mark.parametrize("D,n,T,ppc", CASES[:2])
def test_adjoint_windows_match_oracle(D, n, T, ppc):
    """Loss sum |E^N|^2 after 5 steps, checkpoint windows of 2 steps."""
    from paper_1906_06306_amd import adjoint
    plasma = synth.small_random(D, n, ppc, seed=51 + D, field_amp=0.05, q=0.02)
    nsteps = 5
    L0, o_lx, o_lu, o_lE, o_lB = oracle.adjoint_run(oracle.State(plasma), nsteps)
    sim = make_sim(plasma, T, "fp64")
    ck = adjoint.forward(sim, nsteps, window=2)
    assert sorted(ck) == [0, 2, 4]
    E, B, _ = sim.field_views()
    assert abs(float((E.double() ** 2).sum()) - L0) < 1e-10 * L0
    gl = adjoint.backward(sim, ck, nsteps, 2.0 * E.clone(), torch.zeros_like(B), window=2)
    g_lx, g_lu, g_lE, g_lB = (t.cpu().numpy() for t in gl)
    assert sim.error() == 0
    tol = 1e-10
    assert rel(g_lE, o_lE) < tol and rel(g_lB, o_lB) < tol, (rel(g_lE, o_lE), rel(g_lB, o_lB))
    sl = sim.input_slices()
    for s in range(2):
        a = sl[(0, s)]
        assert rel(g_lx[:, a], o_lx[s]) < tol, (s, rel(g_lx[:, a], o_lx[s]))
        assert rel(g_lu[:, a], o_lu[s]) < tol, (s, rel(g_lu[:, a], o_lu[s]))
    sim.close()


def test_adjoint_requires_tracking():
    from paper_1906_06306_amd import _lib as L
    from paper_1906_06306_amd.sim import PicSim
    plasma = synth.small_random(2, (16, 16), 2, seed=3)
    sim = PicSim(plasma, tile=(8, 8), precision="fp64")
    la, ua, lE, lB = sim.adjoint_buffers()
    assert L.lib().pic_adjoint_step(sim.ctx, la.data_ptr(), ua.data_ptr(), lE.data_ptr(), lB.data_ptr()) \
        == L.PIC_E_STATE
    sim.close()
    sim = make_sim(plasma, (8, 8), "fp64")
    assert L.lib().pic_sort_migrate(sim.ctx, L.PIC_SORT_CELLS) == L.PIC_E_ARG
    assert L.lib().pic_push_interp(sim.ctx, 0) == L.PIC_E_ARG
    sim.close()


# ------------------------------------------------- parameter gradients

def shear_inputs(n, ppc, amp, B0, device):
    """Initial state of the sheared plasma as differentiable tensors of the
    drift amplitude and guide field (thermal part fixed by the seed)."""
    base = synth.shear(n=n, ppc=ppc, amp=0.0, B0=1.0)
    parts = []
    for sp in base.species:
        x = torch.as_tensor(sp.x, device=device)
        u = torch.as_tensor(sp.u, device=device)
        drift = torch.sin(2.0 * math.pi * x[1] / n)
        u = torch.cat([(u[0] + amp * drift)[None], u[1:]], 0)
        parts += [x, u]
    N = n * n
    E0 = torch.zeros((3, N), dtype=torch.float64, device=device)
    zero = torch.zeros(N, dtype=torch.float64, device=device)
    B0f = torch.stack([zero, zero, B0 * torch.ones(N, dtype=torch.float64, device=device)])
    settings = dict(D=2, n=(n, n, 1), c=base.c, charge=[sp.q for sp in base.species],
                    qm=[sp.s for sp in base.species], mass=[sp.m for sp in base.species])
    return settings, E0, B0f, parts


def shear_loss(n, ppc, amp, B0, nsteps, prec, tile, window=8, grad=False):
    from paper_1906_06306_amd.adjoint import PicWindow
    dev = torch.device("cuda:0")
    A = torch.tensor(amp, dtype=torch.float64, device=dev, requires_grad=grad)
    Bz = torch.tensor(B0, dtype=torch.float64, device=dev, requires_grad=grad)
    settings, E0, B0f, parts = shear_inputs(n, ppc, A, Bz, dev)
    settings.update(nsteps=nsteps, window=window, precision=prec, tile=tile)
    E, B = PicWindow.apply(settings, E0, B0f, *parts)
    loss = (E * E).sum()
    if not grad:
        return loss.item()
    loss.backward()
    return loss.item(), A.grad.item(), Bz.grad.item()


def fd_sweep(loss, amp, B0, hs):
    """Central differences in A and B0 for every h of the sweep."""
    out = []
    for h in hs:
        fA = (loss(amp + h, B0) - loss(amp - h, B0)) / (2 * h)
        fB = (loss(amp, B0 + h) - loss(amp, B0 - h)) / (2 * h)
        out.append((h, fA, fB))
    return out


def agrees(g, fds, tol):
    return sum(abs(g - f) <= tol * abs(f) for f in fds) >= 2


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-6), ("fp32", 1e-4)])
def test_parameter_gradients_vs_finite_differences(prec, tol):
    n, ppc, nsteps, tile = 64, 8, 16, (16, 16)
    amp, B0 = 0.1, 0.078772
    print(f"[gpu] shear gradients {prec} n={n} ppc={ppc} steps={nsteps}", flush=True)
    _, gA, gB = shear_loss(n, ppc, amp, B0, nsteps, prec, tile, grad=True)
    sweep = fd_sweep(lambda a, b: shear_loss(n, ppc, a, b, nsteps, "fp64", tile), amp, B0, (1e-7, 1e-8, 1e-9))
    for h, fA, fB in sweep:
        print(f"[gpu] h={h:g}: dL/dA fd {fA:.10e} adjoint {gA:.10e}; dL/dB0 fd {fB:.10e} adjoint {gB:.10e}",
              flush=True)
    assert agrees(gA, [f[1] for f in sweep], tol)
    assert agrees(gB, [f[2] for f in sweep], tol)
