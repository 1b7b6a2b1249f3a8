"""Seeded synthetic plasma states shaped like the paper's workloads.

This module only *generates inputs*: global FP64 particle positions and
four-velocities, initial E and B on the Yee lattice, and the species
constants in code units.  It contains none of the time-step arithmetic;
both the CPU oracle and the HIP path consume what it returns.

Workloads (all self-initialised from formulas; the paper uses no dataset):

* ``weibel``      - 1D3V counter-streaming pair beams (Sect. 5.1 setup,
                    reduced to one dimension along the beams).
* ``turbulence``  - 2D3V decaying magnetised turbulence (Sect. 5.3): warm
                    Maxwell-Juttner pair plasma, guide field B0 z from the
                    magnetisation sigma, 64 random-phase forcing modes.
* ``shock``       - 3D3V pre-shocked pair plasma between conducting walls
                    (Sect. 5.2): hot dense downstream, cold upstream beam.
* ``ensemble``    - many small independent 2D3V thermal boxes.
* ``shear``       - 2D3V magnetised plasma with a sinusoidal shear drift,
                    the differentiable-window workload.

Code units follow App. A: dx = dt = 1, Courant number c, plasma frequency
w_p = c / R_p with R_p the skin depth in cells, |q| = w_p^2 <gamma> /
(N_ppc (1 + m-/m+)), m = |q| for pairs, and B0 from sigma.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.special as sp

BASE_SEED = 190606306


@dataclass
class Species:
    q: float            # macro-particle charge in code units (signed)
    s: float            # App. C factor q/(m m_pm): sign(q)/m_pm
    m: float            # macro-particle mass in code units (|q| m_pm)
    x: np.ndarray       # (D, np) global positions in cells, in [0, n_d)
    u: np.ndarray       # (3, np) four-velocity in units of c


@dataclass
class Plasma:
    D: int
    n: tuple            # (n0, n1, n2), unused dimensions are 1
    c: float            # Courant number
    species: list
    E: np.ndarray       # (3, N) FP64, x fastest
    B: np.ndarray       # (3, N)
    meta: dict = field(default_factory=dict)

    @property
    def ncells(self) -> int:
        return int(self.n[0] * self.n[1] * self.n[2])

    @property
    def nparticles(self) -> int:
        return int(sum(sp_.x.shape[1] for sp_ in self.species))


# --------------------------------------------------------------------------
# Maxwell-Juttner sampling


def mean_gamma_mj(theta: float) -> float:
    """<gamma> of a Maxwell-Juttner distribution at temperature theta,
    K1(1/theta)/K2(1/theta) + 3 theta (exponentially scaled Bessels)."""
    x = 1.0 / theta
    return float(sp.kve(1, x) / sp.kve(2, x) + 3.0 * theta)


def sample_mj(rng: np.random.Generator, theta: float, count: int) -> np.ndarray:
    """Isotropic Maxwell-Juttner four-velocities, shape (3, count).

    Exact rejection sampler in the kinetic energy e = gamma - 1, whose density
    is proportional to (1+e) sqrt(e) sqrt(2+e) exp(-e/theta).  Since
    sqrt(2+e) <= sqrt(2) + sqrt(e), the density is bounded by a mixture of
    Gamma(k, theta) densities with k = 3/2, 2, 5/2, 3 (coefficients sqrt2,
    1, sqrt2, 1); the acceptance probability
    (1+e) sqrt(2+e) / (sqrt2 + sqrt e + sqrt2 e + e^1.5) is >= 1/sqrt(2)
    for every e and theta, so the loop terminates quickly at any
    temperature."""
    shapes = np.array([1.5, 2.0, 2.5, 3.0])
    coef = np.array([math.sqrt(2.0), 1.0, math.sqrt(2.0), 1.0])
    mass = coef * sp.gamma(shapes) * theta ** shapes
    prob = mass / mass.sum()
    out = np.empty(count)
    filled = 0
    while filled < count:
        need = count - filled
        m = int(need * 1.5) + 16
        comp = rng.choice(4, size=m, p=prob)
        e = rng.gamma(shapes[comp], theta)
        se = np.sqrt(e)
        acc = (1.0 + e) * np.sqrt(2.0 + e) / (math.sqrt(2.0) + se + math.sqrt(2.0) * e + e * se)
        keep = e[rng.random(m) < acc][:need]
        out[filled:filled + keep.size] = keep
        filled += keep.size
    gam = 1.0 + out
    pmag = np.sqrt(out * (out + 2.0))          # |u| = sqrt(gamma^2 - 1)
    mu = rng.uniform(-1.0, 1.0, count)
    phi = rng.uniform(0.0, 2.0 * math.pi, count)
    st = np.sqrt(1.0 - mu * mu)
    del gam
    return np.stack([pmag * st * np.cos(phi), pmag * st * np.sin(phi), pmag * mu])


def boost_x(rng: np.random.Generator, u: np.ndarray, gamma_b: float, sign: float) -> np.ndarray:
    """Lorentz boost of rest-frame four-velocities to a drift gamma_b along
    sign*x, with the flux-weighting "flipping" step of Zenitani (2015, Phys.
    Plasmas 22, 042116): a particle whose x-velocity opposes the drift is
    mirrored with probability beta|v'_x| before the boost."""
    beta = sign * math.sqrt(1.0 - 1.0 / gamma_b ** 2)
    g = np.sqrt(1.0 + (u * u).sum(axis=0))
    vx = u[0] / g
    flip = (-beta * vx) > rng.random(u.shape[1])
    ux = np.where(flip, -u[0], u[0])
    out = u.copy()
    out[0] = gamma_b * (ux + beta * g)
    return out


# --------------------------------------------------------------------------
# Unit system (App. A)


def charge_from_skin_depth(c: float, Rp: float, ppc: int, mean_gamma: float,
                           mass_ratio_sum: float = 2.0) -> float:
    """|q| = w_p^2 <gamma> / (N_ppc (1 + m-/m+)) with w_p = c / R_p."""
    wp = c / Rp
    return wp * wp * mean_gamma / (ppc * mass_ratio_sum)


def b0_from_sigma(sigma: float, c: float, ppc: int, qabs: float, mean_gamma: float,
                  mass_ratio_sum: float = 2.0) -> float:
    """B0 from sigma = B0^2 / (N_ppc m c^2 <gamma> (1+m-/m+)), m = |q|."""
    return math.sqrt(sigma * ppc * qabs * c * c * mean_gamma * mass_ratio_sum)


# --------------------------------------------------------------------------
# Layout helpers


def quiet_positions(rng: np.random.Generator, D: int, n: tuple, ppc: int) -> np.ndarray:
    """ppc positions uniform inside every cell, shape (D, ppc*N).  The array is
    ordered layer by layer: layer l holds one particle in each cell, cells in
    x-fastest order."""
    N = int(np.prod(n))
    cells = np.arange(N, dtype=np.int64)
    idx = [cells % n[0], (cells // n[0]) % n[1], cells // (n[0] * n[1])]
    x = np.empty((D, ppc * N))
    for layer in range(ppc):
        sl = slice(layer * N, (layer + 1) * N)
        for d in range(D):
            v = idx[d] + rng.random(N)
            v = np.where(v >= n[d], 0.0, v)
            x[d, sl] = v
    return x


def turbulence_field(rng: np.random.Generator, n: tuple, dB: float, nmodes: int = 8) -> np.ndarray:
    """In-plane perturbation of Sect. 5.3: modes m, n in 1..nmodes with random
    phases and amplitude beta_mn = 2 dB / (N sqrt(m^2+n^2)), realised through
    A_z = sum beta_mn (L/2pi) sin(k_m x + phi) sin(k_n y + psi) on nodes, with
    Bx = A_z(j+1) - A_z(j) and By = -(A_z(i+1) - A_z(i)) on the Yee faces.
    Returns (Bx, By) of shape (2, N); assumes a square n0 x n1 plane."""
    nx, ny = n[0], n[1]
    L = float(nx)
    xs = np.arange(nx, dtype=np.float64)
    ys = np.arange(ny, dtype=np.float64)
    A = np.zeros((ny, nx))
    for mm in range(1, nmodes + 1):
        for nn in range(1, nmodes + 1):
            phi = rng.uniform(0.0, 2.0 * math.pi)
            psi = rng.uniform(0.0, 2.0 * math.pi)
            beta = 2.0 * dB / (nmodes * math.sqrt(mm * mm + nn * nn))
            km = 2.0 * math.pi * mm / L
            kn = 2.0 * math.pi * nn / L
            A += beta * (L / (2.0 * math.pi)) * np.outer(np.sin(kn * ys + psi), np.sin(km * xs + phi))
    Bx = np.roll(A, -1, axis=0) - A
    By = -(np.roll(A, -1, axis=1) - A)
    return np.stack([Bx.reshape(-1), By.reshape(-1)])


def _pair(D, n, c, qabs, xe, ue, xp, up, E, B, meta):
    sp_e = Species(q=-qabs, s=-1.0, m=qabs, x=xe, u=ue)
    sp_p = Species(q=+qabs, s=+1.0, m=qabs, x=xp, u=up)
    return Plasma(D=D, n=tuple(n), c=c, species=[sp_e, sp_p], E=E, B=B, meta=meta)


# --------------------------------------------------------------------------
# Workloads


def weibel(nx: int = 512, ppc: int = 64, gamma_b: float = 3.0, theta: float = 0.01,
           Rp: float = 10.0, c: float = 0.45, seed: int = BASE_SEED + 1, beam_axis: int = 0) -> Plasma:
    """1D3V pair plasma, two counter-streaming beams along x with Lorentz
    factor gamma_b and Maxwell-Juttner spread theta in the beam frame.
    Each species is split half/half between the +x and -x beams; each
    positron sits on an electron (zero initial charge density).

    beam_axis = 1 streams the beams along y instead, across the grid
    direction (the filamentation geometry of Sect. 5.1, where the
    perturbation's wave vector is normal to the beams): the same draws with
    the x and y momentum components exchanged, which leaves the isotropic
    rest-frame spread unchanged."""
    rng = np.random.default_rng(seed)
    n = (nx, 1, 1)
    x = quiet_positions(rng, 1, n, ppc)
    npart = x.shape[1]
    half = npart // 2
    sign = np.where(np.arange(npart) < half, 1.0, -1.0)
    us = []
    for _ in range(2):
        u0 = sample_mj(rng, theta, npart)
        u = np.empty_like(u0)
        u[:, :half] = boost_x(rng, u0[:, :half], gamma_b, +1.0)
        u[:, half:] = boost_x(rng, u0[:, half:], gamma_b, -1.0)
        us.append(u)
    del sign
    if beam_axis not in (0, 1):
        raise ValueError("beam_axis is 0 (beams along x) or 1 (along y)")
    if beam_axis == 1:
        us = [np.ascontiguousarray(u[[1, 0, 2]]) for u in us]
    mg = gamma_b * mean_gamma_mj(theta)
    qabs = charge_from_skin_depth(c, Rp, ppc, mg)
    N = nx
    E = np.zeros((3, N))
    B = np.zeros((3, N))
    meta = dict(workload="weibel", ppc=ppc, theta=theta, gamma_b=gamma_b, Rp=Rp, mean_gamma=mg,
                beam_axis=beam_axis)
    return _pair(1, n, c, qabs, x, us[0], x.copy(), us[1], E, B, meta)


def turbulence(n: int = 1024, ppc: int = 16, theta: float = 0.3, sigma: float = 10.0,
               dB_over_B0: float = 1.0, Rp: float = 3.0, c: float = 0.45,
               nmodes: int = 8, seed: int = BASE_SEED + 2) -> Plasma:
    """2D3V decaying turbulence: thermal pair plasma at rest, guide field
    B0 z from sigma, in-plane forcing modes of amplitude dB = dB_over_B0 B0."""
    rng = np.random.default_rng(seed)
    dims = (n, n, 1)
    x = quiet_positions(rng, 2, dims, ppc)
    ue = sample_mj(rng, theta, x.shape[1])
    up = sample_mj(rng, theta, x.shape[1])
    mg = mean_gamma_mj(theta)
    qabs = charge_from_skin_depth(c, Rp, ppc, mg)
    B0 = b0_from_sigma(sigma, c, ppc, qabs, mg)
    N = n * n
    E = np.zeros((3, N))
    B = np.zeros((3, N))
    B[2, :] = B0
    if dB_over_B0 > 0.0:
        B[0:2] = turbulence_field(rng, dims, dB_over_B0 * B0, nmodes)
    meta = dict(workload="turbulence", ppc=ppc, theta=theta, sigma=sigma, Rp=Rp,
                mean_gamma=mg, B0=B0, dB=dB_over_B0 * B0)
    return _pair(2, dims, c, qabs, x, ue, x.copy(), up, E, B, meta)


def _chunks(total: int, size: int):
    return [(a, min(a + size, total)) for a in range(0, total, size)]


def _run_seeded(seed: int, tasks, fn, workers: int):
    """fn(rng, task) for every task, each with its own generator spawned from
    seed in task order, on a pool of threads (numpy's generators and array
    arithmetic release the interpreter lock).  The results depend on seed and
    on the task list only, not on the order the threads run them."""
    from concurrent.futures import ThreadPoolExecutor
    kids = np.random.SeedSequence(seed).spawn(len(tasks))
    with ThreadPoolExecutor(max_workers=max(1, workers)) as ex:
        list(ex.map(lambda a: fn(np.random.default_rng(a[0]), a[1]), zip(kids, tasks)))


def shock(n: tuple = (1024, 128, 128), x_shock: int = 256, ppc_down: int = 32, ppc_up: int = 8,
          theta_down: float = 3.286, gamma_up: float = 10.0, theta_up: float = 1e-4, Rp: float = 10.0,
          c: float = 0.45, seed: int = BASE_SEED + 3, log=None, workers: int | None = None) -> Plasma:
    """3D3V pre-shocked pair plasma between conducting walls in x (Sect. 5.2
    setup, started from a shocked state): for x < x_shock a hot plasma at
    rest (Maxwell-Juttner theta_down, ppc_down per species, mean Lorentz
    factor equal to the upstream gamma_up), for x >= x_shock the cold
    upstream beam moving towards the wall at x = 0 (Lorentz factor
    gamma_up, theta_up boosted, ppc_up per species).  |q| follows the
    upstream (ppc_up, <gamma> = gamma_up); E = B = 0.  Each positron sits
    on an electron (zero charge density at the start).

    Positions come layer by layer (one particle in every cell per layer,
    the downstream layers first), as quiet_positions lays them out; the
    layers and the four-velocities are drawn in fixed chunks, each from its
    own generator spawned from seed, on `workers` threads (default: up to
    16), so the state depends on the seed alone."""
    import os
    workers = workers or min(16, os.cpu_count() or 1)
    nx, ny, nz = n
    regions = [((x_shock, ny, nz), ppc_down, 0), ((nx - x_shock, ny, nz), ppc_up, x_shock)]
    total = sum(ppc * r[0] * r[1] * r[2] for r, ppc, _ in regions)
    x = np.empty((3, total))
    layers, o = [], 0
    for dims, ppc, x0 in regions:
        N = dims[0] * dims[1] * dims[2]
        cells = np.arange(N, dtype=np.int64)
        idx = [(cells % dims[0]).astype(np.float64), ((cells // dims[0]) % dims[1]).astype(np.float64),
               (cells // (dims[0] * dims[1])).astype(np.float64)]
        for _ in range(ppc):
            layers.append((o, N, dims, idx, x0))
            o += N

    def fill_layer(rng, t):
        o, N, dims, idx, x0 = t
        for d in range(3):
            v = idx[d] + rng.random(N)
            v = np.where(v >= dims[d], 0.0, v)
            x[d, o:o + N] = v + x0 if d == 0 else v

    _run_seeded(seed, layers, fill_layer, workers)
    if log:
        log(f"shock: {total} positions per species")
    nd = ppc_down * x_shock * ny * nz
    step = 1 << 22
    us = []
    for k in range(2):
        u = np.empty((3, total))
        tasks = [(a, b, True) for a, b in _chunks(nd, step)] + \
                [(nd + a, nd + b, False) for a, b in _chunks(total - nd, step)]

        def fill_u(rng, t):
            a, b, down = t
            if down:
                u[:, a:b] = sample_mj(rng, theta_down, b - a)
            else:
                u[:, a:b] = boost_x(rng, sample_mj(rng, theta_up, b - a), gamma_up, -1.0)

        _run_seeded(seed * 4 + 1 + k, tasks, fill_u, workers)
        us.append(u)
        if log:
            log(f"shock: four-velocities of species {k}")
    qabs = charge_from_skin_depth(c, Rp, ppc_up, gamma_up)
    N = nx * ny * nz
    E = np.zeros((3, N))
    B = np.zeros((3, N))
    meta = dict(workload="shock", x_shock=x_shock, ppc_down=ppc_down, ppc_up=ppc_up, theta_down=theta_down,
                gamma_up=gamma_up, theta_up=theta_up, Rp=Rp, walls=True)
    return _pair(3, n, c, qabs, x, us[0], x.copy(), us[1], E, B, meta)


def thermal_box(nx: int, ny: int, ppc: int, theta: float, Rp: float = 3.0, c: float = 0.45,
                seed: int = BASE_SEED + 4) -> Plasma:
    """2D3V thermal pair plasma at rest with no field: one ensemble member."""
    rng = np.random.default_rng(seed)
    dims = (nx, ny, 1)
    x = quiet_positions(rng, 2, dims, ppc)
    ue = sample_mj(rng, theta, x.shape[1])
    up = sample_mj(rng, theta, x.shape[1])
    mg = mean_gamma_mj(theta)
    qabs = charge_from_skin_depth(c, Rp, ppc, mg)
    N = nx * ny
    meta = dict(workload="thermal", ppc=ppc, theta=theta, Rp=Rp, mean_gamma=mg)
    return _pair(2, dims, c, qabs, x, ue, x.copy(), up, np.zeros((3, N)), np.zeros((3, N)), meta)


def ensemble_specs(count: int = 64, seed: int = BASE_SEED + 4):
    """Box sizes, ppc and temperatures of the batched ensemble: sides from
    {64,96,128,192,256} drawn independently, ppc per species from
    {4,8,16,32}, theta log-uniform in [0.01, 1]."""
    rng = np.random.default_rng(seed)
    sides = np.array([64, 96, 128, 192, 256])
    ppcs = np.array([4, 8, 16, 32])
    out = []
    for b in range(count):
        nx = int(rng.choice(sides))
        ny = int(rng.choice(sides))
        ppc = int(rng.choice(ppcs))
        theta = float(10.0 ** rng.uniform(-2.0, 0.0))
        out.append(dict(nx=nx, ny=ny, ppc=ppc, theta=theta, seed=seed * 1000 + b))
    return out


def shear(n: int = 256, ppc: int = 32, theta: float = 0.1, sigma: float = 1.0, amp: float = 0.1,
          Rp: float = 3.0, c: float = 0.45, seed: int = BASE_SEED + 5, B0: float | None = None) -> Plasma:
    """2D3V magnetised pair plasma with a shear drift amp*sin(2 pi y / n) x added to
    every particle's thermal four-velocity; guide field B0 z from sigma unless
    B0 is given."""
    rng = np.random.default_rng(seed)
    dims = (n, n, 1)
    x = quiet_positions(rng, 2, dims, ppc)
    mg = mean_gamma_mj(theta)
    qabs = charge_from_skin_depth(c, Rp, ppc, mg)
    if B0 is None:
        B0 = b0_from_sigma(sigma, c, ppc, qabs, mg)
    drift = amp * np.sin(2.0 * math.pi * x[1] / n)
    ue = sample_mj(rng, theta, x.shape[1])
    up = sample_mj(rng, theta, x.shape[1])
    ue[0] += drift
    up[0] += drift
    N = n * n
    E = np.zeros((3, N))
    B = np.zeros((3, N))
    B[2, :] = B0
    meta = dict(workload="shear", ppc=ppc, theta=theta, sigma=sigma, Rp=Rp, mean_gamma=mg,
                B0=B0, amp=amp)
    return _pair(2, dims, c, qabs, x, ue, x.copy(), up, E, B, meta)


def shear_tensors(base: Plasma, A, B0):
    """The initial state of ``shear`` as torch tensors on the device of the
    0-d tensors A (drift amplitude) and B0 (guide field), through which it
    depends differentiably on both: u_x = u_th,x + A sin(2 pi y / n) for
    both species, B = B0 z, E = 0.  ``base`` is ``shear(..., amp=0)``: it
    supplies positions and the thermal four-velocities.  Returns
    (E (3, N), B (3, N), [x_e, u_e, x_p, u_p])."""
    import torch
    dev = A.device
    n = base.n[0]
    parts = []
    for sp_ in base.species:
        x = torch.as_tensor(sp_.x, device=dev)
        u = torch.as_tensor(sp_.u, device=dev)
        drift = torch.sin(2.0 * math.pi * x[1] / n)
        parts += [x, torch.cat([(u[0] + A * drift)[None], u[1:]], 0)]
    N = base.ncells
    E = torch.zeros((3, N), dtype=torch.float64, device=dev)
    zero = torch.zeros(N, dtype=torch.float64, device=dev)
    B = torch.stack([zero, zero, B0 * torch.ones(N, dtype=torch.float64, device=dev)])
    return E, B, parts


class RecedingInjector:
    """Plasma injected from a wall receding at the speed of light (the
    shock setup of Sect. 5.2): at step k the injector face moves from x0 +
    k c to x0 + (k+1) c, and the slab between the two faces (all y, z) is
    filled with ppc particles per unit cell volume per species, drawn
    uniformly in the slab, moving towards -x with Lorentz factor gamma
    (theta boosted); each positron sits on an electron.  Deterministic per
    (seed, step).  The slab stops at the box end x = n0."""

    def __init__(self, n: tuple, ppc: int, gamma: float, theta: float, c: float = 0.45, x0: float = 0.0,
                 seed: int = BASE_SEED + 6):
        self.n = tuple(n)
        self.D = len(n)
        self.ppc, self.gamma, self.theta, self.c, self.x0, self.seed = ppc, gamma, theta, c, x0, seed
        self._carry = 0.0

    def batch(self, step: int):
        """(x (D, k), u_e (3, k), u_p (3, k)) of the slab of this step
        (steps must be asked in order: the fractional count carries over)."""
        rng = np.random.default_rng([self.seed, step])
        lo = min(self.x0 + step * self.c, self.n[0])
        hi = min(self.x0 + (step + 1) * self.c, self.n[0])
        area = float(np.prod(self.n[1:])) if self.D > 1 else 1.0
        want = self.ppc * (hi - lo) * area + self._carry
        k = int(np.floor(want))
        self._carry = want - k
        x = np.empty((self.D, k))
        x[0] = lo + (hi - lo) * rng.random(k)
        x[0] = np.minimum(x[0], np.nextafter(self.n[0], 0.0))
        for d in range(1, self.D):
            x[d] = self.n[d] * rng.random(k)
            x[d] = np.where(x[d] >= self.n[d], 0.0, x[d])
        ue = boost_x(rng, sample_mj(rng, self.theta, k), self.gamma, -1.0)
        up = boost_x(rng, sample_mj(rng, self.theta, k), self.gamma, -1.0)
        return x, ue, up


def small_random(D: int, n: tuple, ppc: int, theta: float = 0.3, c: float = 0.45,
                 field_amp: float = 0.05, seed: int = 12345, q: float = 1e-3) -> Plasma:
    """A generic small test state: thermal pair plasma plus random E and B of
    amplitude field_amp (no divergence constraint), used for per-kernel
    parity from a common state."""
    rng = np.random.default_rng(seed)
    dims = tuple(n) + (1,) * (3 - len(n))
    x = quiet_positions(rng, D, dims, ppc)
    ue = sample_mj(rng, theta, x.shape[1])
    up = sample_mj(rng, theta, x.shape[1])
    # scramble the order so that tiles hold particles in no particular order
    perm = rng.permutation(x.shape[1])
    xe = x[:, perm]
    perm2 = rng.permutation(x.shape[1])
    xp = x[:, perm2]
    N = int(np.prod(dims))
    E = field_amp * rng.standard_normal((3, N))
    B = field_amp * rng.standard_normal((3, N))
    meta = dict(workload="random", ppc=ppc, theta=theta)
    return _pair(D, dims, c, q, xe, ue, xp, up, E, B, meta)
