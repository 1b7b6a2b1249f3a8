"""The autotuner on the GPU: it times every candidate (tile edge x
work-group size) on the workload itself and returns the fastest; the
configuration it picks then steps the plasma like the oracle."""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_tune_times_every_candidate_and_its_choice_matches_the_oracle():
    from paper_1906_06306_amd import autotune
    from paper_1906_06306_amd.sim import PicSim
    plasma = synth.small_random(2, (64, 32), 8, seed=61, field_amp=0.05)
    print(f"[gpu] autotune 2D 64x32, {plasma.nparticles} particles", flush=True)
    best, res = autotune.tune(plasma, "fp64", blocks=(128, 256), capacity_factor=3.0, steps=2)
    assert set(res) == {(T, b) for T in (8, 16, 32) for b in (128, 256)}
    assert all(v > 0 for v in res.values())
    assert res[best] == min(res.values())
    T, blk = best
    sim = PicSim(plasma, tile=(T, T), precision="fp64", block=blk, capacity_factor=3.0)
    sim.step(2, fused=True, half_b_in_push=True)
    E, B, J = sim.fields_host(0)
    d = sim.diagnostics()
    sim.close()
    st = oracle.State(plasma)
    st.step(2)
    rel = lambda a, b: np.linalg.norm(a - b) / np.linalg.norm(b)
    assert d["status"] == 0
    assert rel(E, st.E) < 1e-12 and rel(J, st.J) < 1e-12 and rel(B, st.B) < 1e-12
