"""The batched ensemble at full size, and the FP64 diagnostics.

* 64 independent 2D3V periodic boxes (sides from {64,...,256}, 4-32
  particles per cell per species, theta from 0.01 to 1; 41.6 M particles)
  stepped together by the persistent tile walker inside a captured HIP
  graph: one replayed step matches the oracle on sampled boxes (the
  smallest, the largest and the first), FP32 tolerance 1e-5, and the
  per-box diagnostics add up to the whole-batch ones.
* pic_diagnostics (FP64 reductions on the GPU) against the oracle's field
  energy, kinetic energy, total charge, Gauss residual and div B of the same
  state, 1e-12 relative.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import tiles

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def common_state(sim, plasma, box):
    st = oracle.State(plasma)
    E, B, _ = sim.fields_host(box)
    st.E[:] = E
    st.B[:] = B
    for s in range(len(plasma.species)):
        tid, xl, u = sim.particles_host(box, s)
        st.x[s] = np.ascontiguousarray(tiles.to_global(tid, xl, plasma.n, sim.T, plasma.D))
        st.u[s] = np.ascontiguousarray(u.astype(np.float64))
    return st


def test_ensemble_graph_persistent_matches_oracle_on_sampled_boxes():
    from paper_1906_06306_amd import _lib as L
    from paper_1906_06306_amd.sim import PicSim
    specs = synth.ensemble_specs()
    boxes = [synth.thermal_box(sp["nx"], sp["ny"], sp["ppc"], sp["theta"], seed=sp["seed"]) for sp in specs]
    npart = sum(b.nparticles for b in boxes)
    print(f"[gpu] ensemble of {len(boxes)} boxes, {npart} particles", flush=True)
    stream = torch.cuda.Stream()
    sim = PicSim(boxes, tile=(16, 16), precision="fp32", capacity_factor=1.5, options=L.PIC_OPT_PERSISTENT,
                 stream=stream)
    sizes = [b.nparticles for b in boxes]
    pick = sorted({0, int(np.argmin(sizes)), int(np.argmax(sizes))})
    assert sim.diagnostics()["particles"] == npart
    sim.capture(1, fused=True, half_b_in_push=True)    # one eager step, then the graph
    # one replayed step from the common state after the eager step
    states = {k: common_state(sim, boxes[k], k) for k in pick}
    for k in pick:
        states[k].step(1)
    sim.replay(1)
    assert sim.error() == 0
    for k in pick:
        E, B, J = sim.fields_host(k)
        st = states[k]
        assert rel(J, st.J) < 1e-5 and rel(E, st.E) < 1e-5 and rel(B, st.B) < 1e-5, \
            (k, rel(J, st.J), rel(E, st.E), rel(B, st.B))
    per = sim.box_diagnostics()
    tot = sim.diagnostics()
    assert sum(d["particles"] for d in per) == tot["particles"] == npart
    assert abs(sum(d["kinetic_energy"] for d in per) - tot["kinetic_energy"]) <= 1e-12 * tot["kinetic_energy"]
    for k in pick:
        uf, uk = states[k].energies()
        assert abs(per[k]["kinetic_energy"] - uk) < 1e-5 * uk
    sim.close()


@pytest.mark.parametrize("D,n,T,ppc", [(1, (96, 1, 1), (16, 1, 1), 24), (2, (48, 32, 1), (16, 16, 1), 6),
                                      (3, (16, 16, 8), (8, 8, 4), 2)])
def test_diagnostics_match_oracle(D, n, T, ppc):
    from paper_1906_06306_amd.sim import PicSim
    plasma = synth.small_random(D, n, ppc, seed=81 + D, field_amp=0.05, q=0.01)
    sim = PicSim(plasma, tile=T, precision="fp64")
    sim.step(3, fused=True, half_b_in_push=True)
    st = common_state(sim, plasma, 0)
    d = sim.diagnostics()
    uf, uk = st.energies()
    assert abs(d["field_energy"] - uf) < 1e-12 * uf
    assert abs(d["kinetic_energy"] - uk) < 1e-12 * uk
    assert d["particles"] == plasma.nparticles
    rho = st.rho()
    assert abs(d["charge_total"] - rho.sum()) < 1e-12 * np.abs(rho).sum()
    g = np.abs(st.gauss_residual()).max()
    assert abs(d["gauss_max"] - g) < 1e-12 * max(g, np.abs(rho).max())
    b = np.abs(st.div_b()).max()
    assert abs(d["divb_max"] - b) < 1e-12 * max(b, np.abs(st.B).max())
    sim.close()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
@pytest.mark.parametrize("D,n,T,ppc", [(1, (96, 1, 1), (16, 1, 1), 24), (2, (48, 32, 1), (16, 16, 1), 6),
                                      (3, (16, 16, 8), (8, 8, 4), 2)])
def test_continuity_residual(D, n, T, ppc, prec, tol):
    """The diagnostics' discrete continuity residual max |rho^{n+1} - rho^n +
    div- J| vanishes to round-off one step after a diagnostics call (App. D's
    charge conservation, measured on the GPU in FP64 from the stored state),
    and is reported as -1 when the calls are not one step apart."""
    from paper_1906_06306_amd.sim import PicSim
    plasma = synth.small_random(D, n, ppc, seed=85 + D, field_amp=0.05, q=0.01)
    sim = PicSim(plasma, tile=T, precision=prec)
    assert sim.diagnostics()["continuity_max"] == -1.0
    sim.step(1, fused=True, half_b_in_push=True)
    d = sim.diagnostics()
    qscale = 0.01 * ppc
    assert 0.0 <= d["continuity_max"] < tol * qscale, d["continuity_max"]
    sim.step(2, fused=True, half_b_in_push=True)
    assert sim.diagnostics()["continuity_max"] == -1.0
    sim.step(1, fused=True, half_b_in_push=True)
    assert 0.0 <= sim.diagnostics()["continuity_max"] < tol * qscale
    sim.close()
