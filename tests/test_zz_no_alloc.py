"""pic_diagnostics_static, the allocation-free diagnostics, against
pic_diagnostics through the C ABI: two identical simulations step in
lockstep, one reports through each entry point; then the same with a
smaller box (fewer tiles: the static array keeps the larger call's
contents beyond what the smaller call writes).  Counts agree exactly; FP64
values to the FP64 bar, 1e-12 relative to the size of what they sum: the
energies relative to themselves, the Gauss and continuity residuals and the
total charge (differences of cancelling charge, whose blocks add FP64
values in LDS in no fixed order, so a recomputation differs in the last
bits) relative to the charge of a node, |q| times the particles per node,
and the total charge times the square root of the node count.  A context
whose tiles need more than the static array is rejected with PIC_E_ARG."""
import ctypes

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def diag_static(sim):
    from paper_1906_06306_amd import _lib as L
    d = L.PicDiag()
    code = L.lib().pic_diagnostics_static(sim.ctx, ctypes.byref(d))
    assert code == 0, (code, L.lib().pic_last_error())
    return dict(field_energy=d.field_energy, kinetic_energy=d.kinetic_energy, gauss_max=d.gauss_max,
                divb_max=d.divb_max, charge_total=d.charge_total, particles=d.particles,
                near_face=d.near_face, error_bits=d.error_bits, continuity_max=d.continuity_max)


def close(a, b, key, rho_scale, ncells):
    if key in ("particles", "near_face", "error_bits"):
        return a == b
    if key == "continuity_max" and (a < 0 or b < 0):
        return a == b
    if key in ("gauss_max", "continuity_max"):
        return abs(a - b) <= 1e-12 * rho_scale
    if key == "charge_total":
        return abs(a - b) <= 1e-12 * rho_scale * ncells ** 0.5
    return abs(a - b) <= 1e-12 * max(abs(a), abs(b))


def compare_runs(plasma, tile, prec, steps):
    from paper_1906_06306_amd.sim import PicSim
    print(f"[gpu] static diagnostics D={plasma.D} n={plasma.n} T={tile} {prec}", flush=True)
    a = PicSim(plasma, tile=tile, precision=prec)
    b = PicSim(plasma, tile=tile, precision=prec)
    ncells = int(np.prod(plasma.n))
    rho_scale = max(abs(s.q) for s in plasma.species) * plasma.nparticles / ncells
    for k in range(steps):
        if k:
            a.step(1, fused=True, half_b_in_push=True)
            b.step(1, fused=True, half_b_in_push=True)
        da = a.diagnostics()
        db = diag_static(b)
        assert da["status"] == 0
        for key in db:
            assert close(da[key], db[key], key, rho_scale, ncells), (k, key, da[key], db[key])
        if k >= 1:
            assert db["continuity_max"] >= 0.0        # one step since the previous call
    a.close()
    b.close()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_static_diagnostics_match_then_smaller_input(prec):
    # larger box first (1,024 tiles), then a smaller one (64 tiles)
    compare_runs(synth.turbulence(n=256, ppc=4, seed=51), (8, 8), prec, 3)
    compare_runs(synth.turbulence(n=64, ppc=4, seed=52), (8, 8), prec, 3)


def test_static_diagnostics_3d():
    compare_runs(synth.small_random(3, (16, 16, 16), 2, seed=53, field_amp=0.02), (8, 8, 8), "fp64", 2)


def test_static_diagnostics_reject_too_many_tiles():
    from paper_1906_06306_amd import _lib as L
    from paper_1906_06306_amd.sim import PicSim
    # 2048 x 512 cells in tiles of 4 x 4: 65,536 tiles x (8 + 25) doubles
    # = 17.3 MB of partials, beyond the 16 MiB array
    plasma = synth.small_random(2, (2048, 512), 1, seed=54)
    sim = PicSim(plasma, tile=(4, 4), precision="fp32", block=64, capacity_factor=2.0)
    d = L.PicDiag()
    code = L.lib().pic_diagnostics_static(sim.ctx, ctypes.byref(d))
    assert code == L.PIC_E_ARG
    assert "static scratch" in L.lib().pic_last_error().decode()
    assert sim.diagnostics()["status"] == 0           # the regular call still works
    sim.close()
