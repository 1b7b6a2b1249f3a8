#!/usr/bin/env python3
"""Throughput of the relativistic PIC step on one MI355X.

Workload: 2D3V decaying relativistic turbulence, 1024 x 1024 periodic cells,
32 x 32 tiles, 16 particles per cell per species (pair plasma, 33.5 M
particles), Maxwell-Juttner theta = 0.3, guide field from sigma = 10,
64 random-phase forcing modes at dB = B0, skin depth 3 cells, Courant 0.45.
One step = the whole hot path: half B update, fused interpolation + Boris
push + ZigZag deposit + tile pack, half B update, current halo fold,
E update with current, tile migration.

Prints ONE JSON line: particle-steps/s of the FP32 path (value), the FP64
path beside it, the roofline of the dominant kernel (the fused push) from
HIP events on its stream, and the FP64 CPU oracle timed on this host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "particle-steps/sec (push+deposit+FDTD) FP32 vs FP64 at 1 GPU; % HBM roofline"

# HBM bytes per launch of the fused push, measured with rocprofv3 --pmc
# FETCH_SIZE and WRITE_SIZE on the turbulence workload and scaled by a plain
# 1 GiB device copy (FETCH x 2.000, WRITE x 1.000), averaged over the first 60
# launches of a run.  Keyed by the code hash of the
# kernel sources they were measured on (kernel_source_hash: file names and
# contents without comments), precision, tile edge, cells per side and
# particles per cell: any other kernel code reports no traffic.
MEASURED_PUSH_TRAFFIC = {
    ("7ea8fa693dd327a3", "fp32", 16, 1024, 16): 1676796437,
    ("7ea8fa693dd327a3", "fp64", 16, 1024, 16): 3200055419,
}

# wave64 VALU instructions per 64 particles of the same push, from rocprofv3
# --pmc SQ_INSTS_VALU over launches 5-39 of a run (same key), and the
# chip's VALU issue peak: 256 CUs x 4 SIMDs, one wave64 instruction per 4
# clocks per SIMD (16 lanes; FP32 not packed) at 2.4 GHz
MEASURED_PUSH_VALU_PER_64 = {
    ("7ea8fa693dd327a3", "fp32", 16, 1024, 16): 387.4,
    ("7ea8fa693dd327a3", "fp64", 16, 1024, 16): 425.3,
}
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4


def strip_comments(src: str) -> str:
    """C/C++ source without comments and with whitespace runs collapsed, so
    that the hash below changes with the code and not with its comments
    (string and character literals are kept as they are)."""
    import re
    tok = re.compile(r'//[^\n]*|/\*.*?\*/|"(?:\\.|[^"\\])*"|\'(?:\\.|[^\'\\])*\'', re.S)
    out = tok.sub(lambda m: " " if m.group(0).startswith("/") else m.group(0), src)
    return " ".join(out.split())


def kernel_source_hash() -> str:
    """Hash of the kernel sources' code (file names, and contents without
    comments), the key of the stored HBM traffic."""
    import glob
    import hashlib
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_1906_06306_amd", "csrc", "*"))):
        h.update(os.path.basename(f).encode())
        with open(f, "r", encoding="utf-8") as fh:
            h.update(strip_comments(fh.read()).encode())
    return h.hexdigest()[:16]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: the workload's run length: turbulence 500, "
                         "ensemble 100, shock 50)")
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=1024, help="cells per side")
    ap.add_argument("--ppc", type=int, default=16, help="particles per cell per species")
    ap.add_argument("--tile", default="auto", help="tile edge, or 'auto' (autotuner over 8/16/32)")
    ap.add_argument("--block", type=int, default=0,
                    help="work-group size of the particle kernels; 0: the autotuner picks 128, 256 or 512 "
                         "(256 when the tile is given)")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--profile-steps", type=int, default=0,
                    help="only run this many fused steps (for rocprofv3), no JSON")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"],
                    help="precision of the --profile-steps and --step-trace runs")
    ap.add_argument("--step-trace", type=int, default=0,
                    help="only run this many fused steps and print every step's kernel times "
                         "(HIP events on the library's stream) as one JSON line, no headline")
    ap.add_argument("--clock-probe", action="store_true",
                    help="with --step-trace: after every step also time a fixed-cycle spin kernel "
                         "(20,000 shader-clock cycles: its duration follows the core clock) and a "
                         "256 MiB device copy (HBM bandwidth)")
    ap.add_argument("--pause-at", type=int, default=0,
                    help="with --step-trace: leave the GPU idle for 3 s before this step")
    ap.add_argument("--capacity", type=float, default=8.0,
                    help="tile segment capacity over the mean count: the turbulent plasma compresses "
                         "16x16-cell tiles to about 4.6 times the mean count within 100 steps")
    ap.add_argument("--cpu-steps", type=int, default=2, help="oracle steps timed for the CPU baseline")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy (to scale rocprofv3 FETCH/WRITE_SIZE)")
    ap.add_argument("--workload", default="turbulence",
                    choices=["turbulence", "shear-adjoint", "shock", "ensemble", "weibel"],
                    help="turbulence: the throughput line; shear-adjoint: the differentiable window "
                         "(256^2, 32 ppc/species, 40 steps, checkpoints every 8) with its forward and "
                         "reverse rates and gradients; shock: 3D3V pre-shocked plasma between walls, "
                         "1024x128x128, 4:1 uneven tiles, per-tile and persistent push; ensemble: 64 "
                         "independent 2D3V boxes stepped together (autotuned tile, persistent walker, graph)")
    ap.add_argument("--fd", action="store_true", help="shear-adjoint: also central differences of the FP64 forward")
    ap.add_argument("--shock-blocks", type=lambda v: [int(b) for b in v.split(",")], default=[256, 512, 1024],
                    help="shock: work-group sizes of the per-tile push to try")
    ap.add_argument("--shock-tile", type=lambda v: tuple(int(b) for b in v.split(",")), default=(8, 8, 8),
                    help="shock: tile edges (x, y, z)")
    ap.add_argument("--pusher", default="boris", choices=["boris", "vay", "hc"],
                    help="turbulence: particle pusher of the timed runs")
    ap.add_argument("--filter-passes", type=int, default=0,
                    help="turbulence: binomial current filter passes per step")
    ap.add_argument("--fdtd-order", type=int, default=2, choices=[2, 4],
                    help="turbulence: FDTD2 (App. B) or FDTD4")
    args = ap.parse_args()
    if args.steps is None:
        args.steps = {"turbulence": 500, "ensemble": 100, "weibel": 200}.get(args.workload, 50)
    return args


def algorithmic_bytes(D, w, n_particles, n_cells):
    """Bytes the step must move: every particle's D positions and 3
    momenta read and written once; E and B (6 words) read and written once
    and J (3 words) written and read once per cell."""
    return n_particles * 2 * (D + 3) * w + n_cells * 18 * w


def push_bytes(D, w, n_particles, n_cells):
    """Bytes the fused push kernel must move per launch: particles read and
    written once, E and B read once, the current written once."""
    return n_particles * 2 * (D + 3) * w + n_cells * 9 * w


def run_gpu(plasma, args, precision, steps, warmup, tile, block=256, profile_only=False):
    import torch
    from paper_1906_06306_amd import _lib as L
    from paper_1906_06306_amd.sim import PicSim

    sim = PicSim(plasma, tile=(tile, tile), precision=precision, block=block,
                 capacity_factor=args.capacity, pusher=args.pusher, filter_passes=args.filter_passes,
                 fdtd_order=args.fdtd_order)
    stream = torch.cuda.current_stream()
    lib = L.lib()
    ctx = sim.ctx

    halfb = args.fdtd_order == 2
    flags = L.PIC_FUSED | (L.PIC_PUSH_HALF_B if halfb else 0)
    fold_e = halfb and not args.filter_passes

    def step(ev=None):
        # the sequence pic_step(flags) enqueues, with events around the
        # fused push
        if not halfb:
            L.check(lib.pic_fdtd_step(ctx, L.PIC_HALF_B))
        if ev is not None:
            ev[0].record(stream)
        L.check(lib.pic_push_interp(ctx, L.PIC_ALL_SPECIES, flags))
        if ev is not None:
            ev[1].record(stream)
        L.check(lib.pic_fdtd_step(ctx, L.PIC_TWO_HALF_B if halfb else L.PIC_HALF_B))
        if fold_e:
            # the fold and E += c curl B - J in one pass
            L.check(lib.pic_deposit_current(ctx, L.PIC_ALL_SPECIES, flags | L.PIC_DEPOSIT_CURL_E))
        else:
            L.check(lib.pic_deposit_current(ctx, L.PIC_ALL_SPECIES, flags))
            if args.filter_passes:
                L.check(lib.pic_filter_current(ctx, args.filter_passes))
            L.check(lib.pic_fdtd_step(ctx, L.PIC_CURL_E_ADD_J))
        L.check(lib.pic_sort_migrate(ctx, 0, None, None, 0))

    if profile_only:
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        code = sim.error()
        sim.close()
        return code

    def spin_us():
        # a kernel that waits 20,000 shader-clock cycles: its duration
        # follows the core clock (outside every timed region)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        torch.cuda._sleep(20000)
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) * 1e3

    torch.cuda._sleep(1000)          # load the spin kernel once, before the warm-up
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    clock = {"spin_20k_cycles_us_before_timed_steps": spin_us()}
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for k in range(steps):
        step(evs[k])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    push_ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    clock["spin_20k_cycles_us_after_timed_steps"] = spin_us()
    # context beside the timed window (not the headline): the same run
    # continued to step 40, then steps 40-60 timed with events, past the
    # slower core clock of the first ~30 ms after the GPU leaves idle
    later = None
    done = warmup + steps
    if done < 40:
        for _ in range(40 - done):
            step()
        ev2 = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
                torch.cuda.Event(enable_timing=True)) for _ in range(20)]
        for e in ev2:
            step((e[0], e[1]))
            e[2].record(stream)
        torch.cuda.synchronize()
        later = {"steps": "40-60", "push_ms": float(np.mean([a.elapsed_time(b) for a, b, _ in ev2])),
                 "ms_per_step_events": float(np.mean([a.elapsed_time(c) for a, _, c in ev2]))}
        clock["spin_20k_cycles_us_after_step_60"] = spin_us()
    sim.diagnostics()
    # one more (untimed) step so that the diagnostics also state the
    # discrete continuity residual of a step
    step()
    diag = sim.diagnostics()
    diag["max_segment_fill"] = sim.fill_ratio()
    sim.close()
    del sim
    torch.cuda.empty_cache()
    return dict(seconds=dt, push_ms=push_ms, diag=diag, later=later, clock=clock)


def valu_roofline(key_hash, prec, tile, args, n_p, push_ms):
    """The push against its VALU issue rate: the measured instructions per
    64 particles for this code, issued in push_ms, over VALU_ISSUE_PEAK
    (null for code without a measurement)."""
    per64 = MEASURED_PUSH_VALU_PER_64.get((key_hash, prec, tile, args.n, args.ppc))
    if per64 is None:
        return None
    achieved = per64 * (n_p / 64.0) / (push_ms * 1e-3)
    return {"bound": "valu_issue", "instr_per_64_particles": per64, "achieved": achieved,
            "peak": VALU_ISSUE_PEAK, "unit": "wave64 instr/s", "frac": achieved / VALU_ISSUE_PEAK,
            "source": "stored: rocprofv3 --pmc SQ_INSTS_VALU of this kernel code on this workload"}


def host_threads() -> int:
    """Host threads the all-thread oracle uses: the CPUs this process may
    run on, at most 16 (one GPU's share of the host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def step_trace(plasma, args, tile, block):
    """Every step's kernel times (us) over args.step_trace fused steps of
    the workload: the push, the two half B updates, the fold with the E
    update, the migration, from HIP events on the library's stream."""
    import torch
    from paper_1906_06306_amd import _lib as L
    from paper_1906_06306_amd.sim import PicSim
    sim = PicSim(plasma, tile=(tile, tile), precision=args.precision, block=block, capacity_factor=args.capacity)
    lib, ctx = L.lib(), sim.ctx
    stream = torch.cuda.current_stream()
    flags = L.PIC_FUSED | L.PIC_PUSH_HALF_B
    probe = args.clock_probe
    if probe:
        src = torch.empty(32 << 20, dtype=torch.float64, device=sim.device)   # 256 MiB
        dst = torch.empty_like(src)
    rows = []
    torch.cuda.synchronize()
    for k in range(args.step_trace):
        if args.pause_at and k == args.pause_at:
            torch.cuda.synchronize()
            time.sleep(3.0)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(7 if probe else 5)]
        ev[0].record(stream)
        L.check(lib.pic_push_interp(ctx, L.PIC_ALL_SPECIES, flags))
        ev[1].record(stream)
        L.check(lib.pic_fdtd_step(ctx, L.PIC_TWO_HALF_B))
        ev[2].record(stream)
        L.check(lib.pic_deposit_current(ctx, L.PIC_ALL_SPECIES, flags | L.PIC_DEPOSIT_CURL_E))
        ev[3].record(stream)
        L.check(lib.pic_sort_migrate(ctx, 0, None, None, 0))
        ev[4].record(stream)
        if probe:
            torch.cuda._sleep(20000)
            ev[5].record(stream)
            dst.copy_(src)
            ev[6].record(stream)
        rows.append(ev)
        if k % 100 == 0:
            log(f"step trace: step {k} enqueued")
    torch.cuda.synchronize()
    t = np.array([[r[i].elapsed_time(r[i + 1]) * 1e3 for i in range(4)] for r in rows])
    status = sim.error()
    sim.close()
    out = {"workload": "turbulence", "precision": args.precision, "tile": tile, "block": block,
           "status": status, "columns": ["push", "two_half_b", "fold_e", "migrate"],
           "us_per_step": [[round(v, 1) for v in row] for row in t.tolist()]}
    if args.pause_at:
        out["idle_3s_before_step"] = args.pause_at
    if probe:
        spin = [r[4].elapsed_time(r[5]) * 1e3 for r in rows]
        cp = [2 * src.numel() * 8 / (r[5].elapsed_time(r[6]) * 1e-3) / 1e9 for r in rows]
        out["spin_20k_cycles_us"] = [round(v, 1) for v in spin]
        out["copy_256MiB_GBs"] = [round(v) for v in cp]
    wins = [(5, 25), (30, 60), (0, len(t)), (100, len(t))]
    if args.pause_at:
        wins += [(args.pause_at - 30, args.pause_at), (args.pause_at + 5, args.pause_at + 25)]
    for a, b in wins:
        if 0 <= a < b <= len(t):
            out[f"mean_steps_{a}_{b}"] = {"push": float(t[a:b, 0].mean()), "step": float(t[a:b].sum(1).mean())}
            if probe:
                out[f"mean_steps_{a}_{b}"]["spin_20k_cycles_us"] = float(np.mean(spin[a:b]))
    print(json.dumps(out), flush=True)


def cpu_oracle_rate(plasma, steps, threads=1):
    """The FP64 oracle, as it stands, on full steps of the same workload, on
    one host thread (orc_step) or on `threads` (orc_step_threads: per-thread
    particle ranges and currents summed in thread order); also returns E, B,
    J after its first step (the reference the GPU paths' one-step error is
    stated against)."""
    import oracle
    st = oracle.State(plasma)
    t0 = time.perf_counter()
    st.step(1, threads=threads)
    t1 = time.perf_counter()
    first = (st.E.copy(), st.B.copy(), st.J.copy())
    t2 = time.perf_counter()
    st.step(steps - 1, threads=threads)
    dt = (t1 - t0) + (time.perf_counter() - t2)
    return plasma.nparticles * steps / dt, dt, first


def common_state_error(plasma, precision, tile, block, warm=5):
    """One GPU step from the GPU's own state after `warm` steps against the
    oracle's step from that state widened to FP64 (whole lattice).  Where the two put
    a particle's end point in different cells (an end point within rounding
    of a face), the oracle deposits from the kernel's end point, so both take
    that integer decision in the kernel's precision; those particles are
    counted and must all be flagged near a face."""
    import torch
    import oracle
    from oracle import tiles
    from paper_1906_06306_amd import _lib as L
    from paper_1906_06306_amd.sim import PicSim
    T = (tile, tile, 1)
    dims = tuple(plasma.n)
    n0 = dims[0]
    sim = PicSim(plasma, tile=(tile, tile), precision=precision, block=block, capacity_factor=3.0,
                 options=L.PIC_OPT_TRACK)
    sim.step(warm, fused=True, half_b_in_push=True)

    def slots(s):
        _, _, _, off, cnt = sim.particle_views()
        off, cnt = off.cpu().numpy(), cnt.cpu().numpy()
        return np.concatenate([np.arange(off[t, s], off[t, s] + cnt[t, s]) for t in range(off.shape[0])])

    st = oracle.State(plasma)
    E0, B0, _ = sim.fields_host(0)
    st.E[:], st.B[:] = E0, B0
    sl0 = []
    for s in range(2):
        tid, xl, u = sim.particles_host(0, s)
        st.x[s] = np.ascontiguousarray(tiles.to_global(tid, xl, dims, T, 2))
        st.u[s] = np.ascontiguousarray(u.astype(np.float64))
        sl0.append(slots(s))
    sim.step(1, fused=True, half_b_in_push=True)
    total, flagged = sim.sort_migrate(flagged_capacity=1 << 22)
    flagged = np.sort(flagged)
    ids = sim.ids_host()
    ends = st.push_particles()
    realigned = unflagged = 0
    for s in range(2):
        tid1, xl1, _ = sim.particles_host(0, s)
        sl1 = slots(s)
        inv = np.full(ids.size, -1, dtype=np.int64)
        inv[sl0[s]] = np.arange(sl0[s].size)
        k = inv[ids[sl1]]
        xg = tiles.to_global(tid1, xl1, dims, T, 2)
        xk = xg + n0 * np.round((ends[s][:, k] - xg) / n0)
        diff = (np.floor(xk) != np.floor(ends[s][:, k])).any(axis=0)
        realigned += int(diff.sum())
        unflagged += int((~np.isin(sl1[diff], flagged)).sum())
        ends[s][:, k[diff]] = xk[:, diff]
    st.finish_step(ends)
    out = {}
    for name, g, r in zip(("E", "B", "J"), sim.fields_host(0), (st.E, st.B, st.J)):
        out[name] = float(np.linalg.norm(g - r) / np.linalg.norm(r))
    out["end_cells_taken_from_kernel"] = realigned
    out["of_them_unflagged"] = unflagged
    out["near_face_flagged"] = int(total)
    out["after_steps"] = warm
    sim.close()
    del sim
    torch.cuda.empty_cache()
    return out


def one_step_error(plasma, precision, tile, ref):
    """Relative L2 of E, B, J after one GPU step from the input state
    against the oracle's first step (input rounding included), and the
    particles flagged near a face before and after it (the ones whose cell,
    and so whose ZigZag relay point, rounding can change)."""
    import torch
    from paper_1906_06306_amd.sim import PicSim
    sim = PicSim(plasma, tile=(tile, tile), precision=precision, capacity_factor=3.0)
    nf0 = sim.diagnostics()["near_face"]
    sim.step(1, fused=True, half_b_in_push=True)
    out = {}
    for name, g, r in zip(("E", "B", "J"), sim.fields_host(0), ref):
        out[name] = float(np.linalg.norm(g - r) / np.linalg.norm(r))
    out["near_face_flagged_at_input"] = int(nf0)
    out["near_face_flagged_after_step"] = int(sim.diagnostics()["near_face"])
    sim.close()
    del sim
    torch.cuda.empty_cache()
    return out


def pick_tile(plasma, args, precision):
    """(tile edge, work-group size, autotuner timings or None)."""
    if args.tile != "auto":
        return int(args.tile), args.block or 256, None
    from paper_1906_06306_amd import autotune
    blocks = (args.block,) if args.block else (128, 256, 512)
    (T, blk), res = autotune.tune(plasma, precision, blocks=blocks, capacity_factor=args.capacity, log=log)
    return T, blk, {f"T{k[0]}_b{k[1]}": round(v * 1e3, 4) for k, v in res.items()}


def copy_bandwidth():
    """GB/s of a plain 1 GiB device-to-device copy (1 GiB read + 1 GiB
    written), the best of 5: the streaming ceiling the push is set against."""
    import torch
    a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    best = 0.0
    for _ in range(6):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        best = max(best, 2 * a.numel() * 4 / (e0.elapsed_time(e1) * 1e-3) / 1e9)
    del a, b
    torch.cuda.empty_cache()
    return best


def calibrate_copy():
    """A plain device copy of 1 GiB (read 1 GiB, write 1 GiB): the reference
    that scales rocprofv3 FETCH_SIZE / WRITE_SIZE to bytes."""
    import torch
    n = 1 << 28
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    log("copy calibration: 3 copies of 1 GiB done")


def bench_adjoint(args):
    """Differentiable window: forward with checkpoints, then the reverse
    sweep (recomputation + adjoint steps), FP32; gradients of sum |E^40|^2 in
    the shear amplitude A and guide field B0."""
    import torch
    import synth
    from paper_1906_06306_amd.adjoint import PicWindow

    # 8^2 tiles: 1,024 work-groups for the 256^2 box (16^2 tiles give only 256)
    n, ppc, nsteps, window, tile = 256, 32, 40, 8, (8, 8)
    amp, B0 = 0.1, 0.078772
    base = synth.shear(n=n, ppc=ppc, amp=0.0, B0=1.0)
    n_p = base.nparticles
    log(f"shear window: {n_p} particles, {nsteps} steps")

    def run(a, b, prec, grad):
        dev = torch.device("cuda:0")
        A = torch.tensor(a, dtype=torch.float64, device=dev, requires_grad=grad)
        Bz = torch.tensor(b, dtype=torch.float64, device=dev, requires_grad=grad)
        E0, B0f, parts = synth.shear_tensors(base, A, Bz)
        settings = dict(D=2, n=base.n, c=base.c, charge=[x.q for x in base.species],
                        qm=[x.s for x in base.species], mass=[x.m for x in base.species], nsteps=nsteps,
                        window=window, precision=prec, tile=tile)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        E, _ = PicWindow.apply(settings, E0, B0f, *parts)
        loss = (E * E).sum()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        if not grad:
            return loss.item(), t1 - t0
        loss.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        return loss.item(), A.grad.item(), Bz.grad.item(), t1 - t0, t2 - t1

    run(amp, B0, "fp32", True)   # warm-up (kernel attributes, allocator)
    L32, gA, gB, tf, tb = run(amp, B0, "fp32", True)
    log(f"fp32: forward {tf:.3f} s, reverse {tb:.3f} s, dL/dA {gA:.8e}, dL/dB0 {gB:.8e}")
    L64, gA64, gB64, tf64, tb64 = run(amp, B0, "fp64", True)
    fd = None
    if args.fd:
        # one-sided differences of the FP64 forward on both sides over a
        # sweep of h; the ZigZag current jumps at face crossings, so only
        # estimates that agree with another interval's are jump-free
        fd = {}
        Lc, _ = run(amp, B0, "fp64", False)
        for key in ("A", "B0"):
            est = []
            for h in (1e-9, 1e-10, 1e-11, 1e-12):
                for sgn in (1.0, -1.0):
                    a1, b1 = (amp + sgn * h, B0) if key == "A" else (amp, B0 + sgn * h)
                    lp, _ = run(a1, b1, "fp64", False)
                    est.append((sgn * h, sgn * (lp - Lc) / h))
            clean = [v for i, (h, v) in enumerate(est)
                     if any(abs(v - w) <= 1e-5 * abs(v) for j, (_, w) in enumerate(est) if j != i)]
            fd[key] = {"estimates": {f"{h:+g}": v for h, v in est}, "jump_free": clean}
    out = {
        "metric": "particle-steps/s of the differentiable window (forward with checkpoints + reverse sweep)",
        "value": n_p * nsteps / (tf + tb),
        "unit": "particle-steps/s",
        "n_gpus": 1, "steps": nsteps, "warmup": 1,
        "ms_per_step": (tf + tb) / nsteps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"2D3V shear {n}x{n}, {ppc} ppc/species, theta=0.1, sigma=1, A=0.1, "
                               f"{nsteps} steps, checkpoints every {window}", "particles": n_p, "tile": tile[0]},
        "forward_s": tf, "reverse_s": tb,
        "forward_rate": n_p * nsteps / tf, "reverse_rate": n_p * nsteps / tb,
        "loss": L32, "dL_dA": gA, "dL_dB0": gB,
        "fp64": {"loss": L64, "dL_dA": gA64, "dL_dB0": gB64, "forward_s": tf64, "reverse_s": tb64},
        "finite_differences_fp64": fd,
    }
    print(json.dumps(out), flush=True)


def bench_shock(args):
    """3D3V pre-shocked pair plasma between conducting walls in x: 1024 x
    128 x 128 cells, 8^3 tiles, 32 ppc/species downstream (x < 256) and 8
    upstream (469.8 M particles), FP32, per-tile push and persistent tile
    walker.  One JSON line (not the headline metric)."""
    import torch
    import synth
    from paper_1906_06306_amd import _lib as L
    from paper_1906_06306_amd.sim import PicSim

    t0 = time.perf_counter()
    plasma = synth.shock(log=log)
    n_p, n_c, D = plasma.nparticles, plasma.ncells, 3
    T = tuple(args.shock_tile)
    log(f"generated {n_p} particles in {time.perf_counter() - t0:.1f}s")
    results = {}
    runs = [(f"per_tile_b{b}", 0, b) for b in args.shock_blocks] + [("persistent", L.PIC_OPT_PERSISTENT, None)]
    for name, opts, blk in runs:
        if blk is None:   # the persistent walker at the best per-tile block size
            blk = int(min((k for k in results), key=lambda k: results[k]["seconds"]).split("_b")[1])
        # segment capacities from the initial per-tile counts (4:1 uneven),
        # with room for the compression at the front
        sim = PicSim(plasma, tile=T, precision="fp32", tile_capacity="auto", capacity_factor=2.0, options=opts,
                     walls=True, block=blk)
        log(f"{name}: initialised")
        stream = torch.cuda.current_stream()
        lib = L.lib()
        flags = L.PIC_FUSED | L.PIC_PUSH_HALF_B
        for _ in range(args.warmup):
            L.check(lib.pic_step(sim.ctx, flags))
        torch.cuda.synchronize()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
        t1 = time.perf_counter()
        for k in range(args.steps):
            evs[k][0].record(stream)
            L.check(lib.pic_push_interp(sim.ctx, L.PIC_ALL_SPECIES, flags))
            evs[k][1].record(stream)
            L.check(lib.pic_fdtd_step(sim.ctx, L.PIC_TWO_HALF_B))
            L.check(lib.pic_deposit_current(sim.ctx, L.PIC_ALL_SPECIES, flags | L.PIC_DEPOSIT_CURL_E))
            L.check(lib.pic_sort_migrate(sim.ctx, 0, None, None, 0))
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        push_ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
        diag = sim.diagnostics()
        sim.close()
        del sim
        torch.cuda.empty_cache()
        results[name] = dict(seconds=dt, push_ms=push_ms, diag=diag, block=blk)
        log(f"{name}: {dt / args.steps * 1e3:.3f} ms/step, push {push_ms:.3f} ms, status {diag['status']}")
    for k, v in results.items():
        if v["diag"]["status"] != 0:
            raise SystemExit(f"device status {v['diag']['status']} after the {k} shock run (capacity or "
                             "numerical error): the measurement is invalid")
    best = min(results, key=lambda k: results[k]["seconds"])
    r = results[best]
    value = n_p * args.steps / r["seconds"]
    pb = push_bytes(D, 4, n_p, n_c)
    achieved = pb / (r["push_ms"] * 1e-3) / 1e9
    out = {
        "metric": "particle-steps/s (push+deposit+FDTD) FP32 at 1 GPU, 3D shock between walls",
        "value": value, "unit": "particle-steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": r["seconds"] / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "3D3V pre-shocked pair plasma 1024x128x128, conducting walls in x, "
                               "x<256: 32 ppc/species theta=3.286; x>=256: 8 ppc/species beam gamma=10",
                   "particles": n_p, "cells": n_c, "tile": list(T), "push": best},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": "k_push<float,3,fused,walls>",
                     "push_ms": r["push_ms"], "algorithmic_bytes_per_launch": pb},
        "step_roofline_frac": algorithmic_bytes(D, 4, n_p, n_c) * value / n_p / 1e9 / HBM_PEAK_GBS,
        "ms_per_step_by_run": {k: v["seconds"] / args.steps * 1e3 for k, v in results.items()},
        "block": r["block"],
        "status": {k: v["diag"]["status"] for k, v in results.items()},
    }
    print(json.dumps(out), flush=True)


def bench_weibel(args):
    """1D3V two-stream (Weibel-shaped) pair plasma, FP64: 512 cells, 64
    ppc/species, the whole 200-step run on the GPU and in the oracle (one
    host thread), with the final fields compared.  Cache-resident (a few MB):
    a rate, no roofline.  One JSON line (not the headline metric)."""
    import torch
    import synth
    import oracle
    from paper_1906_06306_amd import _lib as L
    from paper_1906_06306_amd.sim import PicSim

    plasma = synth.weibel()
    n_p = plasma.nparticles
    flags = L.PIC_FUSED | L.PIC_PUSH_HALF_B
    lib = L.lib()

    def rate(T, steps):
        sim = PicSim(plasma, tile=(T,), precision="fp64", capacity_factor=2.0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            L.check(lib.pic_step(sim.ctx, flags))
        torch.cuda.synchronize()
        sim.close()
        return (time.perf_counter() - t0) / steps

    # tile edge: at 65,536 particles more, smaller segments keep more of the
    # chip busy, against more halo work
    tune = {T: rate(T, 20) for T in ((int(args.tile),) if args.tile != "auto" else (8, 16, 32))}
    T = min(tune, key=tune.get)
    # eager launches; at 65,536 particles a step is a handful of short
    # kernels, so launch overhead counts
    sim = PicSim(plasma, tile=(T,), precision="fp64", capacity_factor=2.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        L.check(lib.pic_step(sim.ctx, flags))
    torch.cuda.synchronize()
    eager_s = time.perf_counter() - t0
    sim.close()
    # the step captured in a HIP graph (capture runs one eager step, then
    # the graph replays the other steps)
    stream = torch.cuda.Stream()
    sim = PicSim(plasma, tile=(T,), precision="fp64", capacity_factor=2.0, stream=stream)
    sim.capture(1, fused=True, half_b_in_push=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.replay(args.steps - 1)
    torch.cuda.synchronize()
    graph_s = (time.perf_counter() - t0) * args.steps / (args.steps - 1)
    gpu_s = min(eager_s, graph_s)
    d = sim.diagnostics()
    E, _, _ = sim.fields_host(0)
    L.check(lib.pic_step(sim.ctx, flags))      # one more step: its continuity residual
    d["continuity_max"] = sim.diagnostics()["continuity_max"]
    sim.close()
    if d["status"] != 0:
        raise SystemExit(f"device status {d['status']} after the Weibel run: the measurement is invalid")
    st = oracle.State(plasma)
    t0 = time.perf_counter()
    st.step(args.steps)
    cpu_s = time.perf_counter() - t0
    nrm = np.linalg.norm(st.E)
    out = {
        "metric": "particle-steps/s (push+deposit+FDTD) FP64 at 1 GPU, 1D two-stream",
        "value": n_p * args.steps / gpu_s, "unit": "particle-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": 0, "ms_per_step": gpu_s / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "1D3V pair plasma, 512 cells, 64 ppc/species, counter-streaming beams gamma=3, "
                               "theta=0.01, c/w_p=10 cells, Courant 0.45", "particles": n_p,
                   "steps": args.steps, "tile": T,
                   "autotune_ms_per_step": {f"T{k}": round(v * 1e3, 4) for k, v in tune.items()}},
        "roofline": None,
        "ms_per_step_eager": eager_s / args.steps * 1e3, "ms_per_step_graph": graph_s / args.steps * 1e3,
        "gauss_max": d["gauss_max"], "continuity_max": d["continuity_max"],
        "field_energy": d["field_energy"],
        "vs_oracle_final_rel_l2_E": float(np.linalg.norm(E - st.E) / (nrm if nrm > 0 else 1.0)),
        "cpu_baseline": {"value": n_p * args.steps / cpu_s, "unit": "particle-steps/s", "cores": 1,
                         "kind": "oracle", "sample": f"the whole {args.steps}-step run, single-threaded FP64 C "
                                                     f"oracle, {cpu_s:.1f} s"},
    }
    print(json.dumps(out), flush=True)


def bench_ensemble(args):
    """64 independent 2D3V thermal boxes of uneven sizes stepped together:
    autotuned tile edge, per-tile launch vs persistent walker, eager vs a
    captured HIP graph; per-box FP64 energies at the start and the end."""
    import torch
    import synth
    from paper_1906_06306_amd import _lib as L
    from paper_1906_06306_amd.sim import PicSim

    specs = synth.ensemble_specs()
    boxes = [synth.thermal_box(sp["nx"], sp["ny"], sp["ppc"], sp["theta"], seed=sp["seed"]) for sp in specs]
    n_p = sum(b.nparticles for b in boxes)
    n_c = sum(b.ncells for b in boxes)
    log(f"ensemble: {len(boxes)} boxes, {n_p} particles, {n_c} cells")
    stream = torch.cuda.Stream()
    flags = L.PIC_FUSED | L.PIC_PUSH_HALF_B
    lib = L.lib()

    def make(T, opts):
        return PicSim(boxes, tile=(T, T), precision="fp32", capacity_factor=1.5, options=opts, stream=stream)

    def timed(sim, steps, graph):
        if graph:
            sim.capture(1, fused=True, half_b_in_push=True)
            run = lambda: L.check(lib.pic_graph_launch(sim.ctx))
        else:
            run = lambda: L.check(lib.pic_step(sim.ctx, flags))
        for _ in range(2):
            run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            run()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    tune = {}
    for T in (8, 16, 32):
        sim = make(T, L.PIC_OPT_PERSISTENT)
        tune[T] = timed(sim, 4, False)
        sim.close()
        log(f"autotune T={T}: {tune[T] * 1e3:.3f} ms/step")
    T = min(tune, key=tune.get)
    modes = {}
    for name, opts, graph in (("per_tile", 0, False), ("persistent", L.PIC_OPT_PERSISTENT, False),
                              ("persistent_graph", L.PIC_OPT_PERSISTENT, True)):
        sim = make(T, opts)
        d0 = sim.box_diagnostics()
        sec = timed(sim, args.steps, graph)
        d1 = sim.box_diagnostics()
        drift = max(abs((b["field_energy"] + b["kinetic_energy"]) - (a["field_energy"] + a["kinetic_energy"]))
                    / (a["field_energy"] + a["kinetic_energy"]) for a, b in zip(d0, d1))
        modes[name] = dict(ms_per_step=sec * 1e3, energy_drift_max=drift,
                           status=max(b["status"] for b in d1))
        sim.close()
        log(f"{name}: {sec * 1e3:.3f} ms/step, max per-box energy drift {drift:.3e}")
    for k, v in modes.items():
        if v["status"] != 0:
            raise SystemExit(f"device status {v['status']} after the {k} ensemble run (capacity or "
                             "numerical error): the measurement is invalid")
    best = min(modes, key=lambda k: modes[k]["ms_per_step"])
    ms = modes[best]["ms_per_step"]
    value = n_p / (ms * 1e-3)
    out = {
        "metric": "particle-steps/s (push+deposit+FDTD) FP32 at 1 GPU, batched ensemble",
        "value": value, "unit": "particle-steps/s", "n_gpus": 1, "steps": args.steps, "warmup": 2,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "64 independent 2D3V thermal pair-plasma boxes, sides in {64..256}, "
                               "4-32 ppc/species, theta 0.01-1", "particles": n_p, "cells": n_c, "tile": T,
                   "mode": best},
        "step_roofline_frac": algorithmic_bytes(2, 4, n_p, n_c) / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "autotune_ms_per_step": {f"T{k}": round(v * 1e3, 4) for k, v in tune.items()},
        "modes": modes,
    }
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU tile decomposition is a design, not a build, here).", file=sys.stderr)
        sys.exit(2)
    import torch
    import synth

    assert torch.cuda.is_available(), "no GPU"
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.workload == "shear-adjoint":
        bench_adjoint(args)
        return
    if args.workload == "shock":
        bench_shock(args)
        return
    if args.workload == "ensemble":
        bench_ensemble(args)
        return
    if args.workload == "weibel":
        bench_weibel(args)
        return
    t0 = time.perf_counter()
    plasma = synth.turbulence(n=args.n, ppc=args.ppc)
    log(f"generated {plasma.nparticles} particles on {args.n}^2 cells in {time.perf_counter() - t0:.1f}s")
    n_p, n_c, D = plasma.nparticles, plasma.ncells, plasma.D
    if args.profile_steps:
        tile = 16 if args.tile == "auto" else int(args.tile)
        code = run_gpu(plasma, args, args.precision, args.profile_steps, 0, tile, args.block or 256, profile_only=True)
        log(f"profile run done, device status {code}")
        return
    if args.step_trace:
        tile = 16 if args.tile == "auto" else int(args.tile)
        step_trace(plasma, args, tile, args.block or 256)
        return
    tile32, blk32, tune32 = pick_tile(plasma, args, "fp32")
    log(f"fp32 run, tile {tile32}, block {blk32}")
    r32 = run_gpu(plasma, args, "fp32", args.steps, args.warmup, tile32, blk32)
    r64 = None
    if not args.no_fp64:
        tile64, blk64, tune64 = pick_tile(plasma, args, "fp64")
        log(f"fp64 run, tile {tile64}, block {blk64}")
        r64 = run_gpu(plasma, args, "fp64", args.steps, args.warmup, tile64, blk64)
    cpu = None
    err32 = err64 = cs32 = cs64 = None
    if not args.no_cpu:
        nth = host_threads()
        log(f"cpu oracle: {args.cpu_steps} full steps on 1 thread")
        rate1, sec1, first = cpu_oracle_rate(plasma, args.cpu_steps)
        log(f"cpu oracle: {args.cpu_steps} full steps on {nth} threads")
        rate_n, sec_n, _ = cpu_oracle_rate(plasma, args.cpu_steps, threads=nth)
        cpu = {"value": rate_n, "unit": "particle-steps/s", "cores": nth, "kind": "oracle",
               "sample": f"{args.cpu_steps} full steps of the same {args.n}^2 workload ({n_p} particles), "
                         f"FP64 C oracle on {nth} host threads (per-thread particle ranges and currents, "
                         f"summed in thread order), {sec_n:.1f} s",
               "single_thread": {"value": rate1, "cores": 1, "seconds": sec1},
               "os_cpu_count": os.cpu_count(), "cpu_model": cpu_model()}
        log("one-step error of the GPU paths against the oracle")
        err32 = one_step_error(plasma, "fp32", tile32, first)
        err64 = one_step_error(plasma, "fp64", tile64 if r64 is not None else tile32, first)
        log("one-step error from the GPU's own state (common state)")
        cs32 = common_state_error(plasma, "fp32", tile32, blk32)
        if r64 is not None:
            cs64 = common_state_error(plasma, "fp64", tile64, blk64)
    for name, r in (("FP32", r32), ("FP64", r64)):
        if r is not None and r["diag"]["status"] != 0:
            # a latched overflow or numerical error: the state, and so the
            # measurement, is invalid
            raise SystemExit(f"device status {r['diag']['status']} after the {name} run (capacity or "
                             "numerical error): the measurement is invalid; raise --capacity")
    value = n_p * args.steps / r32["seconds"]
    pb = push_bytes(D, 4, n_p, n_c)
    achieved = pb / (r32["push_ms"] * 1e-3) / 1e9
    copy_gbs = copy_bandwidth()
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r32["seconds"] / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"2D3V decaying turbulence {args.n}x{args.n} periodic, "
                               f"{args.ppc} ppc/species pair plasma, "
                               "theta=0.3, sigma=10, dB/B0=1 (64 modes), c/w_p=3 cells, Courant 0.45",
                   "particles": n_p, "cells": n_c, "tile": tile32, "block": blk32,
                   "pusher": args.pusher, "filter_passes": args.filter_passes, "fdtd_order": args.fdtd_order,
                   "autotune_ms_per_step": tune32},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": MEASURED_PUSH_TRAFFIC.get((kernel_source_hash(), "fp32", tile32, args.n, args.ppc)),
                     "traffic_source": "stored: rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE of this kernel on this "
                                       "workload, scaled by a plain copy, averaged over 60 launches, for the kernel "
                                       "code with the hash kernel_sources (null for other code)",
                     "kernel": "k_push<float,2,fused>", "push_ms": r32["push_ms"],
                     "algorithmic_bytes_per_launch": pb, "kernel_sources": kernel_source_hash(),
                     "copy_gbs": copy_gbs, "frac_of_copy": achieved / copy_gbs},
        "step_roofline_frac": algorithmic_bytes(D, 4, n_p, n_c) * value / n_p / 1e9 / HBM_PEAK_GBS,
        "valu_roofline": valu_roofline(kernel_source_hash(), "fp32", tile32, args, n_p, r32["push_ms"]),
        "same_run_steps_40_60": r32["later"],
        "clock_probe": r32["clock"],
        "diagnostics_fp32": {k: r32["diag"][k] for k in ("gauss_max", "continuity_max", "divb_max", "field_energy",
                                                         "kinetic_energy", "particles", "near_face",
                                                         "max_segment_fill", "status")},
        "cpu_baseline": cpu,
        "fp32_vs_oracle_1step_rel_l2": err32,
        "fp32_vs_oracle_common_state_rel_l2": cs32,
    }
    if r64 is not None:
        v64 = n_p * args.steps / r64["seconds"]
        pb64 = push_bytes(D, 8, n_p, n_c)
        a64 = pb64 / (r64["push_ms"] * 1e-3) / 1e9
        out["fp64"] = {"value": v64, "ms_per_step": r64["seconds"] / args.steps * 1e3,
                       "push_ms": r64["push_ms"], "speedup_fp32_over_fp64": value / v64,
                       "push_roofline": {"bound": "hbm", "achieved": a64, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                         "frac": a64 / HBM_PEAK_GBS, "algorithmic_bytes_per_launch": pb64,
                                         "traffic": MEASURED_PUSH_TRAFFIC.get((kernel_source_hash(), "fp64", tile64,
                                                                               args.n, args.ppc))},
                       "tile": tile64, "block": blk64, "autotune_ms_per_step": tune64,
                       "gauss_max": r64["diag"]["gauss_max"], "continuity_max": r64["diag"]["continuity_max"],
                       "status": r64["diag"]["status"],
                       "vs_oracle_1step_rel_l2": err64,
                       "valu_roofline": valu_roofline(kernel_source_hash(), "fp64", tile64, args, n_p, r64["push_ms"]),
                       "same_run_steps_40_60": r64["later"],
                       "vs_oracle_common_state_rel_l2": cs64}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
