"""Reverse mode over windows of fused steps, with checkpointed recomputation.

The forward run keeps a copy of the state regions of the workspace (fields,
particle planes, segment counts, origin ids) every ``window`` steps.  The
reverse sweep visits the windows last to first: it restores the window's
checkpoint, re-runs the window while keeping every intermediate state, and
then, step by step backwards, maps the particle adjoints across the step's
migration (``pic_adjoint_unpermute``, from the origin ids the tracked step
recorded) and applies the step's transposed Jacobian (``pic_adjoint_step``).
After the first step the particle adjoints are mapped to the input order
of ``pic_init_tiles``.  All arithmetic runs in the library's kernels; this
module only orders the calls and copies workspaces.

``PicWindow`` wraps one box as a ``torch.autograd.Function`` of its initial
state (positions, four-velocities, E, B), so that gradients of any loss of
the final fields with respect to parameters of the initial state follow
from autograd.
"""
from __future__ import annotations

import torch

from . import _lib as L
from .sim import Box, PicSim

STEP_FLAGS = L.PIC_FUSED | L.PIC_PUSH_HALF_B


def forward(sim: PicSim, nsteps: int, window: int = 8) -> dict:
    """Run nsteps tracked fused steps; return {step: state copy} at the
    window starts."""
    if not sim.cfg.options & L.PIC_OPT_TRACK:
        raise ValueError("the simulation needs options=PIC_OPT_TRACK")
    fn = L.lib().pic_step
    ckpts = {0: sim.snapshot()}
    for k in range(nsteps):
        L.check(fn(sim.ctx, STEP_FLAGS))
        if (k + 1) % window == 0 and k + 1 < nsteps:
            ckpts[k + 1] = sim.snapshot()
    return ckpts


def backward(sim: PicSim, ckpts: dict, nsteps: int, lE, lB, lpos=None, lu=None, window: int = 8):
    """Adjoints of the initial state from those of the state after nsteps.

    lE, lB: (3, cells_total) adjoints of E^N, B^{N-1/2}; lpos, lu: adjoints
    of the final particles in the final state's slots (zero if None).  The
    simulation must hold the final state on entry.  Returns (lpos_in (D,
    n_input), lu_in (3, n_input), lE0, lB0) in the working precision, the
    particle adjoints in the concatenated input order.  Leaves the initial
    state in the workspace."""
    fn = L.lib().pic_step
    la, ua, E_, B_ = sim.adjoint_buffers()
    lb, ub, _, _ = sim.adjoint_buffers()
    lE = lE.to(sim.dtype).contiguous().clone()
    lB = lB.to(sim.dtype).contiguous().clone()
    if lpos is not None:
        la.copy_(lpos)
    if lu is not None:
        ua.copy_(lu)
    cap = int(sim.layout.capacity_total)
    starts = sorted(k for k in ckpts if k < nsteps)
    for w0 in reversed(starts):
        w1 = min(w0 + window, nsteps)
        sim.restore(ckpts[w0])
        states = [ckpts[w0]]
        for j in range(w0, w1):
            L.check(fn(sim.ctx, STEP_FLAGS))
            if j + 1 < w1:                 # the last state stays in the workspace
                states.append(sim.snapshot())
        # Neither the unpermute nor the adjoint step writes the state
        # regions, so the state a reversed step leaves in the workspace (the
        # one before it) is the one the next reversed step starts from.
        for k in range(w1 - 1, w0 - 1, -1):
            lb.zero_()
            ub.zero_()
            sim.unpermute(la, ua, lb, ub, cap)      # from the state after step k
            sim.restore(states[k - w0])
            sim.adjoint_step(lb, ub, lE, lB)        # from the state before it
            la, lb = lb, la
            ua, ub = ub, ua
        del states
    n_in = sim.n_input
    lpos_in = torch.zeros((sim.D, n_in), dtype=sim.dtype, device=sim.device)
    lu_in = torch.zeros((3, n_in), dtype=sim.dtype, device=sim.device)
    sim.unpermute(la, ua, lpos_in, lu_in, n_in)
    return lpos_in, lu_in, lE, lB


class PicWindow(torch.autograd.Function):
    """E^N, B^{N-1/2} of one box after nsteps fused steps, as a function of
    the initial state.  Inputs after the settings: E0 (3, N), B0 (3, N) and
    per species pos (D, np), u (3, np), all FP64 tensors on the device."""

    @staticmethod
    def forward(ctx, settings: dict, E0, B0, *parts):
        ns = len(parts) // 2
        box = Box(D=settings["D"], n=tuple(settings["n"]), c=settings["c"], charge=list(settings["charge"]),
                  qm=list(settings["qm"]), mass=list(settings["mass"]), pos=list(parts[0::2]),
                  u=list(parts[1::2]), E=E0, B=B0)
        sim = PicSim(box, tile=settings["tile"], precision=settings.get("precision", "fp32"),
                     capacity_factor=settings.get("capacity_factor", 2.0), options=L.PIC_OPT_TRACK,
                     device=str(E0.device))
        nsteps, window = int(settings["nsteps"]), int(settings.get("window", 8))
        ckpts = forward(sim, nsteps, window)
        E, B, _ = sim.field_views()
        err = sim.error()
        if err:
            raise L.PicError(err, L.lib().pic_last_error().decode())
        ctx.sim, ctx.ckpts, ctx.nsteps, ctx.window, ctx.ns = sim, ckpts, nsteps, window, ns
        return E.to(torch.float64).clone(), B.to(torch.float64).clone()

    @staticmethod
    def backward(ctx, gE, gB):
        sim = ctx.sim
        z = torch.zeros((3, int(sim.layout.cells_total)), dtype=torch.float64, device=sim.device)
        gE = z if gE is None else gE
        gB = z if gB is None else gB
        lpos, lu, lE, lB = backward(sim, ctx.ckpts, ctx.nsteps, gE, gB, window=ctx.window)
        err = sim.error()
        if err:
            raise L.PicError(err, L.lib().pic_last_error().decode())
        grads = [None, lE.double(), lB.double()]
        for (b, s), sl in sim.input_slices().items():
            grads += [lpos[:, sl].double(), lu[:, sl].double()]
        sim.close()
        ctx.sim = ctx.ckpts = None
        return tuple(grads)
