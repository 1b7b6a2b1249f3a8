"""Thin Python driver over libpic: PyTorch owns the device workspace and the
stream; every step of the method runs in the library's HIP kernels."""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib as L


def _dev64(a, device) -> torch.Tensor:
    """Contiguous FP64 copy of a numpy array or tensor on the device."""
    if isinstance(a, torch.Tensor):
        return a.detach().to(device=device, dtype=torch.float64).contiguous()
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).to(device)


@dataclass
class Box:
    """One periodic box: FP64 global state in code units (App. A)."""
    D: int
    n: tuple                 # (n0, n1, n2)
    c: float
    charge: list             # per species q
    qm: list                 # per species s = q/(m m_pm)
    mass: list               # per species macro-particle mass
    pos: list                # per species (D, np) FP64 global positions
    u: list                  # per species (3, np) FP64 four-velocities
    E: np.ndarray            # (3, N)
    B: np.ndarray            # (3, N)


def box_from_plasma(p) -> Box:
    """Adapter for objects with the attributes of synth.Plasma."""
    return Box(D=p.D, n=tuple(p.n), c=p.c, charge=[s.q for s in p.species], qm=[s.s for s in p.species],
               mass=[s.m for s in p.species], pos=[s.x for s in p.species], u=[s.u for s in p.species],
               E=p.E, B=p.B)


class PicSim:
    """A batch of periodic boxes stepped together on one GPU."""

    def __init__(self, boxes, tile, precision: str = "fp32", block: int = 256, capacity_factor: float = 1.25,
                 tile_capacity=None, outbox_capacity: int = 0, options: int = 0, device: str = "cuda:0",
                 stream=None, walls=False, pusher: str = "boris", filter_passes: int = 0, fdtd_order: int = 2,
                 inject_max: int = 0):
        if not isinstance(boxes, (list, tuple)):
            boxes = [boxes]
        boxes = [b if isinstance(b, Box) else box_from_plasma(b) for b in boxes]
        # settings a re-layout (regrow) repeats
        self._kw = dict(tile=tile, precision=precision, block=block, outbox_capacity=outbox_capacity,
                        options=options, device=device, stream=stream, walls=walls, pusher=pusher,
                        filter_passes=filter_passes, fdtd_order=fdtd_order, inject_max=inject_max)
        self.boxes = boxes
        b0 = boxes[0]
        self.D = b0.D
        self.ns = len(b0.charge)
        self.nb = len(boxes)
        self.c = float(b0.c)
        for b in boxes:
            if b.D != self.D or len(b.charge) != self.ns or float(b.c) != self.c:
                raise ValueError("all boxes must share D, species count and Courant number")
        self.T = tuple(int(t) for t in tile) + (1,) * (3 - len(tile))
        self.prec = L.PIC_FP64 if precision == "fp64" else L.PIC_FP32
        self.dtype = torch.float64 if self.prec == L.PIC_FP64 else torch.float32
        self.device = torch.device(device)
        lib = L.lib()
        # host arrays referenced by the config (kept alive on self)
        self._cells = np.array([list(b.n) + [1] * (3 - len(b.n)) for b in boxes], dtype=np.int32)
        self._charge = np.array([b.charge for b in boxes], dtype=np.float64)
        self._qm = np.array([b.qm for b in boxes], dtype=np.float64)
        self._mass = np.array([b.mass for b in boxes], dtype=np.float64)
        self._counts = np.array([[int(p.shape[1]) for p in b.pos] for b in boxes], dtype=np.int64)
        if isinstance(tile_capacity, str) and tile_capacity == "auto":
            tile_capacity = self._capacity_from_counts(boxes, tile, capacity_factor)
        self._tcap = None if tile_capacity is None else np.ascontiguousarray(tile_capacity, dtype=np.int64)
        cfg = L.PicConfig()
        cfg.dim = self.D
        cfg.precision = self.prec
        cfg.n_species = self.ns
        cfg.n_boxes = self.nb
        for d in range(3):
            cfg.tile[d] = self.T[d]
        cfg.block = block
        cfg.cfl = self.c
        cfg.box_cells = self._cells.ctypes.data
        cfg.charge = self._charge.ctypes.data
        cfg.qm = self._qm.ctypes.data
        cfg.mass = self._mass.ctypes.data
        cfg.tile_capacity = None if self._tcap is None else self._tcap.ctypes.data
        cfg.capacity_factor = capacity_factor
        cfg.outbox_capacity = outbox_capacity
        cfg.options = options
        wl = walls if isinstance(walls, (list, tuple)) else [walls] * self.nb
        self._walls = np.array([L.PIC_WALL_X if w else 0 for w in wl], dtype=np.int32)
        cfg.box_walls = self._walls.ctypes.data if self._walls.any() else None
        cfg.pusher = {"boris": L.PIC_PUSHER_BORIS, "vay": L.PIC_PUSHER_VAY, "hc": L.PIC_PUSHER_HC}[pusher]
        cfg.filter_passes = int(filter_passes)
        cfg.fdtd_order = int(fdtd_order)
        cfg.inject_max = int(inject_max)
        self.cfg = cfg
        lay = L.PicLayout()
        L.check(lib.pic_query(ctypes.byref(cfg), self._counts.ctypes.data, ctypes.byref(lay)))
        self.layout = lay
        self.ws = torch.empty(int(lay.total_bytes) + 256, dtype=torch.uint8, device=self.device)
        base = self.ws.data_ptr()
        self._shift = (-base) % 256
        self.ws_ptr = base + self._shift
        # initial FP64 state, uploaded for the binning kernels
        keep = []
        pos_ptrs, u_ptrs, e_ptrs, b_ptrs = [], [], [], []
        for b in boxes:
            for s in range(self.ns):
                pt = _dev64(b.pos[s], self.device)
                ut = _dev64(b.u[s], self.device)
                keep += [pt, ut]
                pos_ptrs.append(pt.data_ptr())
                u_ptrs.append(ut.data_ptr())
            et = _dev64(b.E, self.device)
            bt = _dev64(b.B, self.device)
            keep += [et, bt]
            e_ptrs.append(et.data_ptr())
            b_ptrs.append(bt.data_ptr())
        n_src = self.nb * self.ns
        self._pos_arr = (ctypes.c_void_p * n_src)(*pos_ptrs)
        self._u_arr = (ctypes.c_void_p * n_src)(*u_ptrs)
        self._e_arr = (ctypes.c_void_p * self.nb)(*e_ptrs)
        self._b_arr = (ctypes.c_void_p * self.nb)(*b_ptrs)
        init = L.PicInitData(self._counts.ctypes.data, ctypes.cast(self._pos_arr, ctypes.c_void_p),
                             ctypes.cast(self._u_arr, ctypes.c_void_p), ctypes.cast(self._e_arr, ctypes.c_void_p),
                             ctypes.cast(self._b_arr, ctypes.c_void_p))
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        ctx = ctypes.c_void_p()
        L.check(lib.pic_init_tiles(ctypes.byref(cfg), self._counts.ctypes.data, ctypes.c_void_p(self.ws_ptr),
                                   int(lay.total_bytes), ctypes.byref(init), ctypes.c_void_p(self.stream.cuda_stream),
                                   ctypes.byref(ctx)))
        self.ctx = ctx
        del keep
        # box geometry on the host for readback
        self.nt = [[b.n[d] // self.T[d] if d < self.D else 1 for d in range(3)] for b in boxes]
        self.tile0 = np.cumsum([0] + [int(np.prod(nt)) for nt in self.nt])[:-1]
        self.cell0 = np.cumsum([0] + [int(np.prod(c)) for c in self._cells])[:-1]

    def _capacity_from_counts(self, boxes, tile, factor):
        """Segment capacities [tiles][species] from the initial particles of
        every tile (uneven loads): ceil(factor * c) + 64, where c is the
        largest count among the tile and its neighbours (a front between a
        dense and a thin region moves into the thin tiles)."""
        T = tuple(int(t) for t in tile) + (1,) * (3 - len(tile))
        out = []
        for b in boxes:
            n = list(b.n) + [1] * (3 - len(b.n))
            nt = [n[d] // T[d] for d in range(3)]
            cols = []
            for pos in b.pos:
                x = pos.detach().cpu().numpy() if isinstance(pos, torch.Tensor) else np.asarray(pos)
                tid = np.zeros(x.shape[1], dtype=np.int64)
                stride = 1
                for d in range(self.D):
                    tid += np.clip(np.floor(x[d] / T[d]).astype(np.int64), 0, nt[d] - 1) * stride
                    stride *= nt[d]
                cnt = np.bincount(tid, minlength=nt[0] * nt[1] * nt[2]).reshape(nt[2], nt[1], nt[0])
                big = cnt.copy()
                for ax in range(3):
                    if nt[2 - ax] > 1:
                        big = np.maximum(big, np.maximum(np.roll(big, 1, axis=ax), np.roll(big, -1, axis=ax)))
                cols.append(big.reshape(-1))
            out.append(np.stack(cols, axis=1))
        return np.ceil(np.concatenate(out, axis=0) * factor).astype(np.int64) + 64

    # ------------------------------------------------------------ calls
    def fdtd(self, phase: int):
        L.check(L.lib().pic_fdtd_step(self.ctx, phase))

    def push(self, fused: bool = True, half_b: bool = False, species=None):
        """interp_em + push of the species in `species` (iterable of
        indices; None: every species)."""
        flags = (L.PIC_FUSED if fused else 0) | (L.PIC_PUSH_HALF_B if half_b else 0)
        L.check(L.lib().pic_push_interp(self.ctx, self._mask(species), flags))

    @staticmethod
    def _mask(species) -> int:
        if species is None:
            return L.PIC_ALL_SPECIES
        m = 0
        for s in species:
            m |= 1 << int(s)
        return m

    def inject(self, box: int, species: int, pos, u):
        """Append particles (FP64 global positions (D, k), four-velocities
        (3, k), numpy or tensors) to box `box`, species `species`."""
        pt = _dev64(pos, self.device)
        ut = _dev64(u, self.device)
        torch.cuda.current_stream(self.device).synchronize()   # inputs resident before the library's stream reads them
        L.check(L.lib().pic_inject(self.ctx, int(box), int(species), int(pt.shape[1]), pt.data_ptr(), ut.data_ptr()))
        self.stream.synchronize()                              # keep the inputs alive until binned

    def filter_current(self, passes: int):
        L.check(L.lib().pic_filter_current(self.ctx, int(passes)))

    def deposit(self, species=None, curl_e: bool = False):
        flags = L.PIC_DEPOSIT_CURL_E if curl_e else 0
        L.check(L.lib().pic_deposit_current(self.ctx, self._mask(species), flags))

    def sort_migrate(self, sort_cells: bool = False, counts: bool = False, flagged_capacity: int = -1):
        """Particle communication (and the cell sort).  counts=True returns
        the migration counts [tiles][species][3^D] (int32 numpy);
        flagged_capacity >= 0 also returns (total, slots) of the particles
        flagged near a cell face afterwards."""
        mc = fl = None
        if counts:
            mc = torch.zeros(int(self.layout.tiles_total) * self.ns * 3 ** self.D, dtype=torch.int32,
                             device=self.device)
        if flagged_capacity >= 0:
            fl = torch.full((flagged_capacity + 1,), -1, dtype=torch.int64, device=self.device)
        # the outputs are written on the library's stream
        torch.cuda.current_stream(self.device).synchronize()
        L.check(L.lib().pic_sort_migrate(self.ctx, L.PIC_SORT_CELLS if sort_cells else 0,
                                         None if mc is None else mc.data_ptr(),
                                         None if fl is None else fl.data_ptr(), max(flagged_capacity, 0)))
        if mc is None and fl is None:
            return None
        self.stream.synchronize()
        out = []
        if mc is not None:
            out.append(mc.view(-1, self.ns, 3 ** self.D).cpu().numpy())
        if fl is not None:
            h = fl.cpu().numpy()
            n = int(h[0])
            out.append((n, h[1:1 + min(n, flagged_capacity)]))
        return out[0] if len(out) == 1 else tuple(out)

    def step(self, n: int = 1, fused: bool = True, sort_cells: bool = False, half_b_in_push: bool = False):
        flags = ((L.PIC_FUSED if fused else 0) | (L.PIC_SORT_CELLS if sort_cells else 0)
                 | (L.PIC_PUSH_HALF_B if half_b_in_push else 0))
        fn = L.lib().pic_step
        for _ in range(n):
            L.check(fn(self.ctx, flags))

    def capture(self, nsteps: int = 1, fused: bool = True, sort_cells: bool = False,
                half_b_in_push: bool = True):
        """Capture nsteps steps into a HIP graph (after one eager step)."""
        flags = ((L.PIC_FUSED if fused else 0) | (L.PIC_SORT_CELLS if sort_cells else 0)
                 | (L.PIC_PUSH_HALF_B if half_b_in_push else 0))
        L.check(L.lib().pic_graph_capture(self.ctx, nsteps, flags))

    def replay(self, n: int = 1):
        fn = L.lib().pic_graph_launch
        for _ in range(n):
            L.check(fn(self.ctx))

    # ------------------------------------------------------ reverse mode
    def _state_ranges(self):
        """Byte ranges of the workspace that hold the state between steps:
        E, B, positions, four-velocities, segment counts, the error word and
        (with origin tracking) the origin ids.  Everything else is constant
        tables or scratch that the next step rewrites."""
        lay = self.layout
        w = int(lay.elem_bytes)
        N = int(lay.cells_total)
        cap = int(lay.capacity_total)
        nts = int(lay.tiles_total) * self.ns
        r = [(lay.off_E, 3 * N * w), (lay.off_B, 3 * N * w), (lay.off_pos, self.D * cap * w),
             (lay.off_u, 3 * cap * w), (lay.off_seg_count, nts * 4), (lay.off_error, 4)]
        if self.cfg.options & L.PIC_OPT_TRACK:
            r.append((lay.off_ids, cap * 4))
        r.sort()
        merged = []
        for off, n in r:
            off = int(off)
            if merged and off - (merged[-1][0] + merged[-1][1]) <= 256:
                merged[-1][1] = off + n - merged[-1][0]
            else:
                merged.append([off, n])
        return [(self._shift + off, n) for off, n in merged]

    def snapshot(self) -> list:
        """Copy of the state regions of the workspace (see _state_ranges)."""
        return [self.ws[a:a + n].clone() for a, n in self._state_ranges()]

    def restore(self, snap: list):
        for (a, n), t in zip(self._state_ranges(), snap):
            self.ws[a:a + n].copy_(t)

    def adjoint_buffers(self):
        """Zeroed particle and field adjoint arrays in the state layout."""
        cap = int(self.layout.capacity_total)
        N = int(self.layout.cells_total)
        z = lambda *shape: torch.zeros(shape, dtype=self.dtype, device=self.device)
        return z(self.D, cap), z(3, cap), z(3, N), z(3, N)

    @property
    def n_input(self) -> int:
        return int(self._counts.sum())

    def unpermute(self, lpos_a, lu_a, lpos_b, lu_b, stride: int):
        for t in (lpos_a, lu_a, lpos_b, lu_b):
            assert t.dtype == self.dtype and t.is_contiguous() and t.device == self.device
        assert lpos_b.shape[-1] == stride and lu_b.shape[-1] == stride
        L.check(L.lib().pic_adjoint_unpermute(self.ctx, lpos_a.data_ptr(), lu_a.data_ptr(), lpos_b.data_ptr(),
                                              lu_b.data_ptr(), int(stride)))

    def adjoint_step(self, lpos, lu, lE, lB):
        for t in (lpos, lu, lE, lB):
            assert t.dtype == self.dtype and t.is_contiguous() and t.device == self.device
        L.check(L.lib().pic_adjoint_step(self.ctx, lpos.data_ptr(), lu.data_ptr(), lE.data_ptr(), lB.data_ptr()))

    def input_slices(self):
        """(box, species) -> slice of the concatenated input order."""
        out, o = {}, 0
        for b in range(self.nb):
            for s in range(self.ns):
                c = int(self._counts[b, s])
                out[(b, s)] = slice(o, o + c)
                o += c
        return out

    def ids_view(self) -> torch.Tensor:
        """The origin ids (int32 per particle slot, `PIC_OPT_TRACK`) as a
        device view of the workspace: after init the index in the
        concatenated input, after a step the slot the particle held before
        it."""
        if not self.cfg.options & L.PIC_OPT_TRACK:
            raise ValueError("origin ids need options=PIC_OPT_TRACK")
        return self._view(self.layout.off_ids, int(self.layout.capacity_total), torch.int32)

    def ids_host(self):
        torch.cuda.synchronize(self.device)
        return self.ids_view().cpu().numpy()

    def error(self) -> int:
        code = L.lib().pic_error(self.ctx)
        return code

    def diagnostics(self) -> dict:
        d = L.PicDiag()
        code = L.lib().pic_diagnostics(self.ctx, ctypes.byref(d))
        if code not in (0,) and code < (1 << 8):
            L.check(code)
        return dict(field_energy=d.field_energy, kinetic_energy=d.kinetic_energy, gauss_max=d.gauss_max,
                    divb_max=d.divb_max, charge_total=d.charge_total, particles=d.particles,
                    near_face=d.near_face, error_bits=d.error_bits, continuity_max=d.continuity_max,
                    status=code)

    def box_diagnostics(self) -> list:
        """Diagnostics of every box (FP64), one dict per box."""
        arr = (L.PicDiag * self.nb)()
        code = L.lib().pic_diagnostics_boxes(self.ctx, ctypes.cast(arr, ctypes.c_void_p))
        if code not in (0,) and code < (1 << 8):
            L.check(code)
        return [dict(field_energy=d.field_energy, kinetic_energy=d.kinetic_energy, gauss_max=d.gauss_max,
                     divb_max=d.divb_max, charge_total=d.charge_total, particles=d.particles,
                     error_bits=d.error_bits, continuity_max=d.continuity_max, status=code) for d in arr]

    def close(self):
        if getattr(self, "ctx", None):
            L.lib().pic_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ----------------------------------------------------------- views
    def _view(self, off: int, count: int, dtype) -> torch.Tensor:
        esize = torch.empty((), dtype=dtype).element_size()
        start = self._shift + int(off)
        return self.ws[start:start + count * esize].view(dtype)

    def field_views(self):
        N = int(self.layout.cells_total)
        E = self._view(self.layout.off_E, 3 * N, self.dtype).view(3, N)
        B = self._view(self.layout.off_B, 3 * N, self.dtype).view(3, N)
        J = self._view(self.layout.off_J, 3 * N, self.dtype).view(3, N)
        return E, B, J

    def fill_ratio(self) -> float:
        """Largest count / capacity over the (tile, species) segments: the
        headroom left before a push or migration would latch
        PIC_E_CAPACITY."""
        nts = int(self.layout.tiles_total) * self.ns
        cap = self._view(self.layout.off_seg_capacity, nts, torch.int32).float()
        cnt = self._view(self.layout.off_seg_count, nts, torch.int32).float()
        return float((cnt / cap).max().item())

    def particle_views(self):
        cap = int(self.layout.capacity_total)
        pos = self._view(self.layout.off_pos, self.D * cap, self.dtype).view(self.D, cap)
        u = self._view(self.layout.off_u, 3 * cap, self.dtype).view(3, cap)
        xold = self._view(self.layout.off_xold, self.D * cap, self.dtype).view(self.D, cap)
        nts = int(self.layout.tiles_total) * self.ns
        off = self._view(self.layout.off_seg_offset, nts, torch.int64).view(-1, self.ns)
        cnt = self._view(self.layout.off_seg_count, nts, torch.int32).view(-1, self.ns)
        return pos, u, xold, off, cnt

    def fields_host(self, box: int = 0):
        """E, B, J of one box as FP64 numpy arrays (3, N)."""
        torch.cuda.synchronize(self.device)
        E, B, J = self.field_views()
        a = int(self.cell0[box])
        n = int(np.prod(self._cells[box]))
        return tuple(t[:, a:a + n].double().cpu().numpy() for t in (E, B, J))

    def particles_host(self, box: int = 0, species: int = 0, with_xold: bool = False):
        """Particles of one box and species in storage order (tiles in id
        order): (tile_id (np,), x_loc (D, np) in the working precision,
        u (3, np)[, xold (D, np)])."""
        torch.cuda.synchronize(self.device)
        pos, u, xold, off, cnt = self.particle_views()
        off = off.cpu().numpy()
        cnt = cnt.cpu().numpy()
        t0 = int(self.tile0[box])
        ntb = int(np.prod(self.nt[box]))
        idx, tid = [], []
        for t in range(t0, t0 + ntb):
            o, c = int(off[t, species]), int(cnt[t, species])
            idx.append(np.arange(o, o + c))
            tid.append(np.full(c, t - t0, dtype=np.int64))
        idx = np.concatenate(idx) if idx else np.zeros(0, dtype=np.int64)
        tid = np.concatenate(tid) if tid else np.zeros(0, dtype=np.int64)
        it = torch.as_tensor(idx, device=self.device)
        out = [tid, pos[:, it].cpu().numpy(), u[:, it].cpu().numpy()]
        if with_xold:
            out.append(xold[:, it].cpu().numpy())
        return tuple(out)

    def state_boxes(self) -> list:
        """The current state as FP64 `Box` objects, particles in storage
        order.  Exact: a tile-local coordinate in the working precision plus
        its tile centre (an integer) is an FP64 sum without rounding, and
        binning that global position gives back the same tile and local
        coordinate."""
        out = []
        for i, b in enumerate(self.boxes):
            E, B, _ = self.fields_host(i)
            pos, us = [], []
            for s in range(self.ns):
                tid, xl, u = self.particles_host(i, s)
                nt = self.nt[i]
                tc = [tid % nt[0], (tid // nt[0]) % nt[1], tid // (nt[0] * nt[1])]
                x = np.empty((self.D, tid.size))
                for d in range(self.D):
                    x[d] = tc[d] * self.T[d] + self.T[d] // 2 + xl[d].astype(np.float64)
                pos.append(x)
                us.append(u.astype(np.float64))
            out.append(Box(D=b.D, n=tuple(b.n), c=b.c, charge=list(b.charge), qm=list(b.qm), mass=list(b.mass),
                           pos=pos, u=us, E=E, B=B))
        return out

    def regrow(self, factor: float = 2.0) -> "PicSim":
        """A new simulation holding this one's state, with segment capacities
        of factor x the current counts (dilated over neighbouring tiles, as
        `tile_capacity="auto"`).  For runs whose plasma compresses beyond the
        capacities chosen at the start (`fill_ratio` tells the headroom).  A
        host round trip of the whole state: meant for occasional use.  The
        caller closes the old simulation.  Origin ids (`PIC_OPT_TRACK`) do not
        carry over, so tracked runs are refused."""
        if self.cfg.options & L.PIC_OPT_TRACK:
            raise ValueError("origin ids do not carry over a re-layout")
        kw = dict(self._kw)
        kw.update(tile_capacity="auto", capacity_factor=factor)
        return PicSim(self.state_boxes(), **kw)

    def counts_host(self):
        torch.cuda.synchronize(self.device)
        _, _, _, _, cnt = self.particle_views()
        return cnt.cpu().numpy()
