"""Launch-shape autotuner: times candidate tile edges and work-group sizes on
the actual workload and keeps the fastest.

Tile size matters for the method (the paper reports a 2x spread in wall time
between tile sizes for one run, Sect. 6 footnote); on gfx950 the trade-off is
LDS per work-group (fields, halo and the 8-byte current block grow as T^D)
against halo overhead and the number of work-groups.
"""
from __future__ import annotations

import time

import torch

from . import _lib as L
from .sim import PicSim


def time_step(sim: PicSim, steps: int = 4, warmup: int = 2, flags: int = L.PIC_FUSED | L.PIC_PUSH_HALF_B) -> float:
    """Seconds per step of the fused step on the sim's stream."""
    fn = L.lib().pic_step
    for _ in range(warmup):
        L.check(fn(sim.ctx, flags))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        L.check(fn(sim.ctx, flags))
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def lds_bytes(D: int, T: int, elem: int) -> int:
    """LDS of the fused push for edge T: E (T+3)^D, B (T+2)^D, 8-byte J (T+3)^D."""
    return 3 * (T + 3) ** D * elem + 3 * (T + 2) ** D * elem + 3 * (T + 3) ** D * 8


def candidates(plasma, elem: int):
    """Tile edges that divide every box side and fit the 160 KB of LDS."""
    D = plasma.D
    sides = [plasma.n[d] for d in range(D)]
    out = []
    for T in (8, 16, 32):
        if all(s % T == 0 for s in sides) and lds_bytes(D, T, elem) <= 160 * 1024:
            out.append(T)
    return out


def tune(plasma, precision: str = "fp32", blocks=(256,), capacity_factor: float = 2.0, steps: int = 4,
         log=None):
    """Return (best (T, block), {(T, block): seconds per step})."""
    elem = 8 if precision == "fp64" else 4
    edges = candidates(plasma, elem)
    if not edges:
        raise ValueError(f"no tile edge of 8, 16 or 32 divides every side of {tuple(plasma.n[:plasma.D])} "
                         "and fits the LDS; give the tile explicitly")
    results = {}
    for T in edges:
        for blk in blocks:
            sim = PicSim(plasma, tile=(T,) * plasma.D, precision=precision, block=blk,
                         capacity_factor=capacity_factor)
            sec = time_step(sim, steps=steps)
            sim.close()
            del sim
            torch.cuda.empty_cache()
            results[(T, blk)] = sec
            if log:
                log(f"autotune {precision} T={T} block={blk}: {sec * 1e3:.3f} ms/step")
    best = min(results, key=results.get)
    return best, results
