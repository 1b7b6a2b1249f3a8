"""Plain FP64 CPU oracle of the relativistic PIC step (arXiv 1906.06306).

TEST INFRASTRUCTURE ONLY: only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the HIP implementation in ``paper_1906_06306_amd``; both consume the
seeded inputs of ``synth``.

``pic_oracle.c`` holds the arithmetic (global periodic arrays, Table-1 order,
double precision, no FMA contraction); this module is argument marshalling
plus the tile-level integer rules in :mod:`oracle.tiles`.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pic_oracle.c")
_LIB = os.path.join(_HERE, "_build", "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc -O2 -ffp-contract=off."""
    os.makedirs(os.path.dirname(_LIB), exist_ok=True)
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                               "-shared", "-Wall", "-pthread", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I = ctypes.c_int
        I64 = ctypes.c_int64
        Dbl = ctypes.c_double
        sig = {
            "orc_advance_b": (None, [I, P, Dbl, P, P]),
            "orc_advance_e": (None, [I, P, Dbl, P, P]),
            "orc_add_current": (None, [P, P, P]),
            "orc_interp": (None, [I, P, P, P, I64, P, P, P]),
            "orc_interp_walls": (None, [I, P, P, P, I64, P, P, P]),
            "orc_boris": (None, [I64, Dbl, Dbl, P, P, P]),
            "orc_move": (None, [I, I64, Dbl, P, P, P]),
            "orc_zigzag": (None, [I, P, Dbl, I64, P, P, P, P]),
            "orc_wrap": (None, [I, P, I64, P]),
            "orc_step": (I, [I, P, Dbl, I, P, P, P, P, P, P, P, P]),
            "orc_step_walls": (I, [I, P, Dbl, I, P, P, P, P, P, P, P, P]),
            "orc_step_opts": (I, [I, P, Dbl, I, P, P, P, P, P, P, P, P, I, I, I, I]),
            "orc_advance_b4": (None, [I, P, Dbl, P, P]),
            "orc_advance_e4": (None, [I, P, Dbl, P, P]),
            "orc_vay": (None, [I64, Dbl, Dbl, P, P, P]),
            "orc_hc": (None, [I64, Dbl, Dbl, P, P, P]),
            "orc_filter_binomial": (I, [I, P, I, I, P]),
            "orc_rho": (None, [I, P, Dbl, I64, P, P]),
            "orc_div_edge": (None, [P, P, P]),
            "orc_div_face": (None, [P, P, P]),
            "orc_field_energy": (Dbl, [P, P, P]),
            "orc_kinetic_energy": (Dbl, [I64, Dbl, Dbl, P]),
            "orc_step_adjoint": (I, [I, P, Dbl, I, P, P, P, P, P, P, P, P, P, P, P]),
            "orc_step_threads": (I, [I, P, Dbl, I, P, P, P, P, P, P, P, P, I]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.dtype == np.float64 or a.dtype == np.int32 or a.dtype == np.int64, a.dtype
    assert a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.c_void_p)


def _dims(n) -> np.ndarray:
    return np.ascontiguousarray(np.array(list(n) + [1] * (3 - len(n)), dtype=np.int32))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


# ------------------------------------------------------------------ fields

def advance_b(D, n, h, E, B):
    """B -= h curl+(E) (in place on B)."""
    dims = _dims(n)
    lib().orc_advance_b(D, _p(dims), float(h), _p(E), _p(B))


def advance_e(D, n, h, B, E):
    """E += h curl-(B) (in place on E)."""
    dims = _dims(n)
    lib().orc_advance_e(D, _p(dims), float(h), _p(B), _p(E))


def advance_b4(D, n, h, E, B):
    """B -= h curl+(E), fourth-order differences (in place on B)."""
    dims = _dims(n)
    lib().orc_advance_b4(D, _p(dims), float(h), _p(E), _p(B))


def advance_e4(D, n, h, B, E):
    """E += h curl-(B), fourth-order differences (in place on E)."""
    dims = _dims(n)
    lib().orc_advance_e4(D, _p(dims), float(h), _p(B), _p(E))


def add_current(n, J, E):
    dims = _dims(n)
    lib().orc_add_current(_p(dims), _p(J), _p(E))


# --------------------------------------------------------------- particles

def interp(D, n, E, B, x, walls: bool = False):
    x = _f64(x)
    np_ = x.shape[1]
    Ep = np.zeros((3, np_))
    Bp = np.zeros((3, np_))
    dims = _dims(n)
    fn = lib().orc_interp_walls if walls else lib().orc_interp
    fn(D, _p(dims), _p(_f64(E)), _p(_f64(B)), np_, _p(x), _p(Ep), _p(Bp))
    return Ep, Bp


def boris(c, s, Ep, Bp, u):
    """u (3, np) updated in place."""
    lib().orc_boris(u.shape[1], float(c), float(s), _p(_f64(Ep)), _p(_f64(Bp)), _p(u))


def vay(c, s, Ep, Bp, u):
    """Vay pusher; u (3, np) updated in place."""
    lib().orc_vay(u.shape[1], float(c), float(s), _p(_f64(Ep)), _p(_f64(Bp)), _p(u))


def higuera_cary(c, s, Ep, Bp, u):
    """Higuera-Cary pusher; u (3, np) updated in place."""
    lib().orc_hc(u.shape[1], float(c), float(s), _p(_f64(Ep)), _p(_f64(Bp)), _p(u))


def filter_binomial(D, n, passes, F):
    """passes of the 3-point binomial filter on F (planes, N) in place."""
    dims = _dims(n)
    F2 = F.reshape(-1, int(np.prod(dims)))
    assert F2.flags.c_contiguous and F2.dtype == np.float64
    if lib().orc_filter_binomial(D, _p(dims), int(passes), F2.shape[0], _p(F2)) != 0:
        raise MemoryError("oracle filter could not allocate scratch")


def move(D, c, u, x):
    """x (D, np) advanced in place; returns the (3, np) displacement."""
    disp = np.zeros((3, u.shape[1]))
    lib().orc_move(D, u.shape[1], float(c), _p(u), _p(x), _p(disp))
    return disp


def zigzag(D, n, q, x1, x2, disp, J):
    dims = _dims(n)
    lib().orc_zigzag(D, _p(dims), float(q), x1.shape[1], _p(_f64(x1)), _p(_f64(x2)),
                     _p(_f64(disp)), _p(J))


def wrap(D, n, x):
    dims = _dims(n)
    lib().orc_wrap(D, _p(dims), x.shape[1], _p(x))


def rho(D, n, q, x, out=None):
    dims = _dims(n)
    N = int(np.prod(dims))
    if out is None:
        out = np.zeros(N)
    lib().orc_rho(D, _p(dims), float(q), x.shape[1], _p(_f64(x)), _p(out))
    return out


def div_edge(n, F):
    dims = _dims(n)
    out = np.zeros(int(np.prod(dims)))
    lib().orc_div_edge(_p(dims), _p(_f64(F)), _p(out))
    return out


def div_face(n, F):
    dims = _dims(n)
    out = np.zeros(int(np.prod(dims)))
    lib().orc_div_face(_p(dims), _p(_f64(F)), _p(out))
    return out


def field_energy(n, E, B):
    dims = _dims(n)
    return lib().orc_field_energy(_p(dims), _p(_f64(E)), _p(_f64(B)))


def kinetic_energy(mass, c, u):
    return lib().orc_kinetic_energy(u.shape[1], float(mass), float(c), _p(_f64(u)))


# -------------------------------------------------------------- full step

class State:
    """Mutable FP64 copy of a synth.Plasma for stepping with the oracle."""

    def __init__(self, plasma):
        self.D = plasma.D
        self.n = tuple(plasma.n)
        self.c = float(plasma.c)
        self.E = _f64(plasma.E).copy()
        self.B = _f64(plasma.B).copy()
        self.J = np.zeros_like(self.E)
        self.x = [_f64(s.x).copy() for s in plasma.species]
        self.u = [_f64(s.u).copy() for s in plasma.species]
        self.q = [float(s.q) for s in plasma.species]
        self.s = [float(s.s) for s in plasma.species]
        self.m = [float(s.m) for s in plasma.species]

    def step(self, nsteps: int = 1, walls: bool = False, pusher: int = 0, filter_passes: int = 0,
             fdtd_order: int = 2, threads: int = 1):
        """nsteps full steps; walls=True: conducting, reflecting walls at
        x = 0 and x = n0 (y, z periodic), else periodic everywhere; pusher
        0 Boris, 1 Vay, 2 Higuera-Cary; filter_passes binomial passes on J;
        fdtd_order 2 or 4.  threads > 1 (periodic Boris/FDTD2 step only):
        the particle rows on that many host threads, per-thread currents
        summed in thread order."""
        if threads > 1:
            if walls or pusher or filter_passes or fdtd_order != 2:
                raise ValueError("the threaded step covers the periodic Boris/FDTD2 step")
            fn = lambda *a: lib().orc_step_threads(*a, int(threads))
        elif pusher or filter_passes or fdtd_order != 2:
            extra = (int(walls), int(pusher), int(filter_passes), int(fdtd_order))
            fn = lambda *a: lib().orc_step_opts(*a, *extra)
        else:
            fn = lib().orc_step_walls if walls else lib().orc_step
        ns = len(self.x)
        dims = _dims(self.n)
        n_per = np.array([x.shape[1] for x in self.x], dtype=np.int64)
        xp = (ctypes.c_void_p * ns)(*[x.ctypes.data for x in self.x])
        up = (ctypes.c_void_p * ns)(*[u.ctypes.data for u in self.u])
        q = np.array(self.q, dtype=np.float64)
        s = np.array(self.s, dtype=np.float64)
        for _ in range(nsteps):
            rc = fn(self.D, _p(dims), self.c, ns, _p(n_per),
                                ctypes.cast(xp, ctypes.c_void_p), ctypes.cast(up, ctypes.c_void_p),
                                _p(q), _p(s), _p(self.E), _p(self.B), _p(self.J))
            if rc != 0:
                raise MemoryError("oracle step could not allocate scratch")

    def push_particles(self):
        """First half of one periodic Boris/FDTD2 step, with the routines
        and in the order of orc_step: push_half_b1, then interp_em and push
        of every species.  Returns the unwrapped end points x^{n+1} (one
        (D, np) array per species); finish_step completes the step."""
        self._x1 = [x.copy() for x in self.x]
        self._disp = []
        advance_b(self.D, self.n, 0.5 * self.c, self.E, self.B)
        ends = []
        for s in range(len(self.x)):
            Ep, Bp = interp(self.D, self.n, self.E, self.B, self.x[s])
            boris(self.c, self.s[s], Ep, Bp, self.u[s])
            x2 = np.ascontiguousarray(self.x[s].copy())
            self._disp.append(move(self.D, self.c, self.u[s], x2))
            ends.append(x2)
        return ends

    def finish_step(self, ends):
        """Second half of the step begun by push_particles: push_half_b2,
        push_e, comp_curr from the start points to `ends` (the end points
        push_particles returned, or the same points with some replaced by a
        caller that takes a cell decision in another precision), the wrap
        and add_cur."""
        advance_b(self.D, self.n, 0.5 * self.c, self.E, self.B)
        advance_e(self.D, self.n, self.c, self.B, self.E)
        self.J[:] = 0.0
        for s in range(len(self.x)):
            x2 = np.ascontiguousarray(ends[s], dtype=np.float64)
            zigzag(self.D, self.n, self.q[s], self._x1[s], x2, self._disp[s], self.J)
            wrap(self.D, self.n, x2)
            self.x[s] = x2
        add_current(self.n, self.J, self.E)
        del self._x1, self._disp

    def append(self, species: int, x, u):
        """Add particles (global x (D, k), u (3, k)) after the existing ones:
        particle creation, the oracle side of the injector."""
        self.x[species] = np.ascontiguousarray(np.concatenate([self.x[species], _f64(x)], axis=1))
        self.u[species] = np.ascontiguousarray(np.concatenate([self.u[species], _f64(u)], axis=1))

    def copy(self):
        other = State.__new__(State)
        other.D, other.n, other.c = self.D, self.n, self.c
        other.E, other.B, other.J = self.E.copy(), self.B.copy(), self.J.copy()
        other.x = [x.copy() for x in self.x]
        other.u = [u.copy() for u in self.u]
        other.q, other.s, other.m = list(self.q), list(self.s), list(self.m)
        return other

    def step_adjoint(self, lx, lu, lE, lB):
        """Reverse one step taken from this state: lx, lu (per species) and
        lE, lB (fields) hold the adjoints of the step's outputs on entry and
        the adjoints of this state on exit (all modified in place)."""
        ns = len(self.x)
        dims = _dims(self.n)
        n_per = np.array([x.shape[1] for x in self.x], dtype=np.int64)
        arr = lambda lst: (ctypes.c_void_p * ns)(*[a.ctypes.data for a in lst])
        xp, up, lxp, lup = arr(self.x), arr(self.u), arr(lx), arr(lu)
        q = np.array(self.q, dtype=np.float64)
        s = np.array(self.s, dtype=np.float64)
        rc = lib().orc_step_adjoint(self.D, _p(dims), self.c, ns, _p(n_per),
                                    ctypes.cast(xp, ctypes.c_void_p), ctypes.cast(up, ctypes.c_void_p),
                                    _p(q), _p(s), _p(self.E), _p(self.B),
                                    ctypes.cast(lxp, ctypes.c_void_p), ctypes.cast(lup, ctypes.c_void_p),
                                    _p(lE), _p(lB))
        if rc != 0:
            raise MemoryError("oracle adjoint could not allocate scratch")

    def rho(self):
        out = np.zeros(int(np.prod(_dims(self.n))))
        for x, q in zip(self.x, self.q):
            rho(self.D, self.n, q, x, out)
        return out

    def gauss_residual(self):
        return div_edge(self.n, self.E) - self.rho()

    def hold_walls(self):
        """Zero the wall planes (Ey, Ez, Bx at i = 0) of the fields."""
        N = int(np.prod(_dims(self.n)))
        n0 = self.n[0]
        idx = np.arange(0, N, n0)
        self.E[1, idx] = 0.0
        self.E[2, idx] = 0.0
        self.B[0, idx] = 0.0

    def div_b(self):
        return div_face(self.n, self.B)

    def energies(self):
        uf = field_energy(self.n, self.E, self.B)
        uk = sum(kinetic_energy(m, self.c, u) for m, u in zip(self.m, self.u))
        return uf, uk


def loss_e2(st) -> float:
    """L = sum over cells of |E|^2."""
    return float(np.sum(st.E * st.E))


def adjoint_run(st0, nsteps: int):
    """Loss sum |E^N|^2 after nsteps from state st0 (not modified) and its
    adjoints with respect to st0: returns (L, lx, lu, lE, lB).  Keeps every
    intermediate state (for small systems)."""
    states = [st0.copy()]
    for _ in range(nsteps):
        nxt = states[-1].copy()
        nxt.step(1)
        states.append(nxt)
    fin = states[-1]
    L = loss_e2(fin)
    lE = 2.0 * fin.E.copy()
    lB = np.zeros_like(fin.B)
    lx = [np.zeros_like(x) for x in fin.x]
    lu = [np.zeros_like(u) for u in fin.u]
    for k in range(nsteps - 1, -1, -1):
        states[k].step_adjoint(lx, lu, lE, lB)
    return L, lx, lu, lE, lB
