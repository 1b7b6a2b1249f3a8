"""GPU Vay and Higuera-Cary pushers and the binomial current filter against
the oracle (one fused step from a common state; E, B, J within 1e-12 / 1e-5
relative L2, every particle matched through its origin id), the filter
entry point against the oracle's filter, and the option combinations the
library rejects."""
import numpy as np
import pytest

import oracle
import synth
from oracle import tiles

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5}
PUSHER = {"boris": 0, "vay": 1, "hc": 2}


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def slots_in_order(sim, species):
    _, _, _, off, cnt = sim.particle_views()
    off, cnt = off.cpu().numpy(), cnt.cpu().numpy()
    return np.concatenate([np.arange(off[t, species], off[t, species] + cnt[t, species])
                           for t in range(off.shape[0])])


def common_state(sim, plasma):
    st = oracle.State(plasma)
    E, B, _ = sim.fields_host(0)
    st.E[:] = E
    st.B[:] = B
    for s in range(len(plasma.species)):
        tid, xl, u = sim.particles_host(0, s)
        st.x[s] = np.ascontiguousarray(tiles.to_global(tid, xl, plasma.n, sim.T, plasma.D))
        st.u[s] = np.ascontiguousarray(u.astype(np.float64))
    return st


CASES = [
    (1, (64, 1, 1), (16, 1, 1), 16),
    (2, (32, 24, 1), (8, 8, 1), 6),
    (3, (16, 8, 8), (8, 4, 4), 2),
]


def check_step(D, n, T, ppc, prec, pusher, passes, walls, seed, order=2):
    from paper_1906_06306_amd import _lib as L
    from paper_1906_06306_amd.sim import PicSim
    plasma = synth.small_random(D, n, ppc, theta=1.0, seed=seed, field_amp=0.2, q=0.01)
    print(f"[gpu] D={D} {prec} pusher={pusher} passes={passes} walls={walls} order={order}", flush=True)
    sim = PicSim(plasma, tile=T, precision=prec, capacity_factor=2.0, options=L.PIC_OPT_TRACK, walls=walls,
                 pusher=pusher, filter_passes=passes, fdtd_order=order)
    st = common_state(sim, plasma)
    if walls:
        st.hold_walls()
    pre = [slots_in_order(sim, s) for s in range(2)]
    sim.step(1, fused=True, half_b_in_push=True)
    st.step(1, walls=walls, pusher=PUSHER[pusher], filter_passes=passes, fdtd_order=order)
    assert sim.error() == 0
    tol = TOL[prec]
    E, B, J = sim.fields_host(0)
    assert rel(J, st.J) < tol and rel(E, st.E) < tol and rel(B, st.B) < tol, (rel(J, st.J), rel(E, st.E))
    ids = sim.ids_host()
    for s in range(2):
        tid, xl, u = sim.particles_host(0, s)
        k = np.searchsorted(pre[s], ids[slots_in_order(sim, s)])
        gx = tiles.to_global(tid, xl, n, T, D)
        d = np.abs(gx - st.x[s][:, k])
        for dd in range(1 if walls else 0, D):
            d[dd] = np.minimum(d[dd], n[dd] - d[dd])
        assert d.max() < (1e-12 if prec == "fp64" else 4e-6 * max(T))
        assert rel(u.astype(np.float64), st.u[s][:, k]) < 10 * tol
    sim.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("pusher", ["vay", "hc"])
@pytest.mark.parametrize("D,n,T,ppc", CASES)
def test_pushers_match_oracle(D, n, T, ppc, pusher, prec):
    check_step(D, n, T, ppc, prec, pusher, 0, False, 91 + D)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("D,n,T,ppc", CASES)
def test_filtered_step_matches_oracle(D, n, T, ppc, prec):
    check_step(D, n, T, ppc, prec, "boris", 3, False, 95 + D)


@pytest.mark.parametrize("D,n,T,ppc", CASES)
def test_walls_with_higuera_cary(D, n, T, ppc):
    check_step(D, n, T, ppc, "fp64", "hc", 0, True, 97 + D)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("D,n,T,ppc", CASES)
def test_fdtd4_step_matches_oracle(D, n, T, ppc, prec):
    check_step(D, n, T, ppc, prec, "hc", 8, False, 99 + D, order=4)


@pytest.mark.parametrize("D,n,T,m", [(1, (32, 1, 1), (16, 1, 1), (5, 0, 0)),
                                     (3, (16, 12, 8), (8, 4, 4), (2, 3, 1))])
def test_fdtd4_plane_wave_on_gpu(D, n, T, m):
    """Vacuum FDTD4 on the GPU follows the exact fourth-order discrete plane
    wave for 300 steps (FP64, 1e-12)."""
    import math
    from paper_1906_06306_amd.sim import PicSim
    c = 0.45
    k = np.array([2 * math.pi * m[d] / n[d] if d < D else 0.0 for d in range(3)])
    kap = 2 * (9.0 / 8.0 * np.sin(k / 2) - 1.0 / 24.0 * np.sin(3 * k / 2))
    w = 2 * math.asin(c * np.linalg.norm(kap) / 2)
    e = np.array([0.3, 1.0, -0.4])
    e = e - kap * (e @ kap) / (kap @ kap)
    b = c * np.cross(kap, e) / (2 * math.sin(w / 2))
    stag = np.array([[0.5, 0, 0], [0, 0.5, 0], [0, 0, 0.5], [0, 0.5, 0.5], [0.5, 0, 0.5], [0.5, 0.5, 0]])
    N = int(np.prod(n))
    ci = np.arange(N)
    idx = np.stack([ci % n[0], (ci // n[0]) % n[1], ci // (n[0] * n[1])]).astype(float)

    def wave(t):
        E = np.stack([e[q] * np.cos(k @ (idx + stag[q][:, None]) - w * t) for q in range(3)])
        B = np.stack([b[q] * np.cos(k @ (idx + stag[3 + q][:, None]) - w * (t - 0.5)) for q in range(3)])
        return E, B
    p = synth.small_random(D, n[:D], 1, seed=1)
    for sp in p.species:
        sp.x = sp.x[:, :0].copy()
        sp.u = sp.u[:, :0].copy()
    p.E, p.B = wave(0)
    sim = PicSim(p, tile=T[:D], precision="fp64", fdtd_order=4)
    sim.step(300, fused=True, half_b_in_push=True)
    E, B, _ = sim.fields_host(0)
    Ea, Ba = wave(300)
    assert rel(E, Ea) < 1e-12 and rel(B, Ba) < 1e-12, (rel(E, Ea), rel(B, Ba))
    sim.close()


@pytest.mark.parametrize("passes", [1, 2, 8])
def test_filter_entry_point_matches_oracle(passes):
    from paper_1906_06306_amd.sim import PicSim
    plasma = synth.small_random(2, (48, 32), 2, seed=7, field_amp=0.05)
    sim = PicSim(plasma, tile=(16, 16), precision="fp64")
    rng = np.random.default_rng(passes)
    _, _, Jv = sim.field_views()
    J0 = rng.standard_normal(tuple(Jv.shape))
    Jv.copy_(torch.as_tensor(J0, device=Jv.device))
    sim.filter_current(passes)
    _, _, J = sim.fields_host(0)
    ref = J0.copy()
    oracle.filter_binomial(2, (48, 32), passes, ref)
    assert np.abs(J - ref).max() < 1e-14 * np.abs(ref).max()
    sim.close()


def test_rejected_combinations():
    from paper_1906_06306_amd import _lib as L
    from paper_1906_06306_amd.sim import PicSim
    plasma = synth.small_random(2, (16, 16), 2, seed=3)
    with pytest.raises(L.PicError):
        PicSim(plasma, tile=(8, 8), precision="fp64", walls=True, filter_passes=2)
    sim = PicSim(plasma, tile=(8, 8), precision="fp64", options=L.PIC_OPT_TRACK, pusher="vay")
    la, ua, lE, lB = sim.adjoint_buffers()
    assert L.lib().pic_adjoint_step(sim.ctx, la.data_ptr(), ua.data_ptr(), lE.data_ptr(), lB.data_ptr()) \
        == L.PIC_E_ARG
    sim.close()
    sim = PicSim(plasma, tile=(8, 8), precision="fp64", walls=True)
    assert L.lib().pic_filter_current(sim.ctx, 2) == L.PIC_E_ARG
    sim.close()
    with pytest.raises(L.PicError):
        PicSim(plasma, tile=(8, 8), precision="fp64", walls=True, fdtd_order=4)
    sim = PicSim(plasma, tile=(8, 8), precision="fp64", fdtd_order=4)
    assert L.lib().pic_push_interp(sim.ctx, L.PIC_ALL_SPECIES, L.PIC_FUSED | L.PIC_PUSH_HALF_B) == L.PIC_E_ARG
    sim.close()
