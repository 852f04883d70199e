"""Seeded synthetic inputs for the Vlasov-hybrid time step.

This module only *draws* initial marker populations; it holds none of the
method's arithmetic (no weighting, no moments, no field solve, no push).  Both
the GPU path and the CPU oracle take their inputs from here, so a parity test
compares the two on bit-identical marker arrays.

Marker loading follows the paper's simple strategy (Sec. 2, the paragraphs on
marker weights; Sec. 3.1, marker creation): the same number of markers
(``ppc``) is placed in every phase-space cell and each marker carries the value
of the initial distribution at its own position, f_l = f0(x_l, v_l).

Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014): state advances by the golden
gamma 0x9E3779B97F4A7C15 and each output is the finalising mix of the state;
a uniform double is (z >> 11) * 2**-53.  The n-th output of a stream seeded with
``seed`` is therefore mix(seed + (n + 1) * gamma), which is evaluated here in
vectorised form.

Draw order within one stream: first the phases of the perturbation modes (one
draw each), then, marker by marker in velocity-major order (for each velocity
cell, for each x cell, for each of the ppc markers), one draw for the in-cell x
offset followed by one per velocity component, and finally (stress variant
only) one draw per marker for a log-uniform weight.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Sequence

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, start: int, count: int) -> np.ndarray:
    """Outputs ``start .. start+count-1`` of the SplitMix64 stream for ``seed``."""
    with np.errstate(over="ignore"):
        n = np.arange(start + 1, start + 1 + count, dtype=np.uint64)
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + n * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniforms(seed: int, start: int, count: int) -> np.ndarray:
    """Uniform doubles in [0, 1) from the SplitMix64 stream (53-bit)."""
    z = splitmix64(seed, start, count)
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


@dataclasses.dataclass(frozen=True)
class Population:
    """One drifting Maxwellian in every velocity component: density * prod_d M(v_d; u_d, s_d)."""
    density: float
    drift: tuple = (0.0, 0.0, 0.0)
    vth: tuple = (1.0, 1.0, 1.0)


@dataclasses.dataclass(frozen=True)
class Workload:
    """A synthetic plasma: phase-space grid, species constants and initial f0.

    Units are normalised (q = -1, m = 1, Poisson constant c_P = 1, so the
    electron plasma frequency and Debye length are 1 for unit density and
    thermal speed); the paper's CGS form is c_P = 4*pi.
    """
    name: str
    vdim: int
    nx: int
    nv: tuple
    L: float
    vmin: tuple
    vmax: tuple
    ppc: int
    dt: float
    steps: int
    seed: int
    populations: tuple
    # density perturbation 1 + sum_m amp_m * cos(k_m x + phi_m); phases are
    # drawn from the stream when ``random_phases`` is set, else all zero.
    mode_numbers: tuple = ()
    mode_amplitude: float = 0.0
    random_phases: bool = False
    weights: str = "analytic"   # or "logu": f_l log-uniform in [1e-8, 1]
    q: float = -1.0
    m: float = 1.0
    c_p: float = 1.0
    first_kick: int = 0
    B: tuple = (0.0, 0.0, 0.0)      # uniform background magnetic field (1D-3V)

    @property
    def n_markers(self) -> int:
        return self.nx * int(np.prod(self.nv[: self.vdim])) * self.ppc

    @property
    def n_cells(self) -> int:
        return self.nx * int(np.prod(self.nv[: self.vdim]))

    @property
    def dx(self) -> float:
        return self.L / self.nx

    def dv(self, d: int = 0) -> float:
        return (self.vmax[d] - self.vmin[d]) / self.nv[d]

    def replace(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)


def _maxwellian(v: np.ndarray, u: float, s: float) -> np.ndarray:
    return np.exp(-((v - u) ** 2) / (2.0 * s * s)) / (s * math.sqrt(2.0 * math.pi))


def mode_phases(w: Workload) -> np.ndarray:
    if not w.mode_numbers:
        return np.zeros(0)
    if w.random_phases:
        return 2.0 * math.pi * uniforms(w.seed, 0, len(w.mode_numbers))
    return np.zeros(len(w.mode_numbers))


def f0(w: Workload, x: np.ndarray, v: Sequence[np.ndarray]) -> np.ndarray:
    """Initial distribution at arbitrary phase points (x, v_0[, v_1, v_2])."""
    k1 = 2.0 * math.pi / w.L
    dens = np.ones_like(x)
    for mnum, ph in zip(w.mode_numbers, mode_phases(w)):
        dens = dens + w.mode_amplitude * np.cos(k1 * mnum * x + ph)
    g = np.zeros_like(x)
    for p in w.populations:
        term = np.full_like(x, p.density)
        for d in range(w.vdim):
            term = term * _maxwellian(v[d], p.drift[d], p.vth[d])
        g = g + term
    return dens * g


def _n_pre(w: Workload) -> int:
    return len(w.mode_numbers) if w.random_phases else 0


def markers(w: Workload, row_begin: int = 0, row_end: int | None = None):
    """Markers of velocity rows [row_begin, row_end) as FP64 SoA arrays.

    A "row" is one velocity cell (the flattened (jz, jy, jx) index in 1D-3V).
    Returns (x[n], v[vdim, n], f[n]) in velocity-major generation order.
    """
    nrows = int(np.prod(w.nv[: w.vdim]))
    if row_end is None:
        row_end = nrows
    per_row = w.nx * w.ppc
    n = (row_end - row_begin) * per_row
    nd = 1 + w.vdim
    first = row_begin * per_row
    u = uniforms(w.seed, _n_pre(w) + first * nd, n * nd).reshape(n, nd)
    loc = np.arange(first, first + n, dtype=np.int64)
    cell = loc // w.ppc
    i = cell % w.nx
    row = cell // w.nx
    dx = w.dx
    x = (i.astype(np.float64) + u[:, 0]) * dx
    x = np.where(x >= w.L, x - w.L, x)
    v = np.empty((w.vdim, n))
    rem = row.copy()
    for d in range(w.vdim):
        j = rem % w.nv[d]
        rem //= w.nv[d]
        v[d] = w.vmin[d] + (j.astype(np.float64) + u[:, 1 + d]) * w.dv(d)
    if w.weights == "logu":
        uf = uniforms(w.seed, _n_pre(w) + w.n_markers * nd + first, n)
        f = 10.0 ** (-8.0 + 8.0 * uf)
    else:
        f = f0(w, x, v)
    return x, v, f


def markers_threaded(w: Workload, threads: int | None = None, block_rows: int | None = None):
    """Same arrays as ``markers(w)``, drawn by a pool of threads over blocks of
    velocity rows (numpy releases the interpreter lock inside its kernels), for
    the large configurations."""
    import os
    from concurrent.futures import ThreadPoolExecutor
    nrows = int(np.prod(w.nv[: w.vdim]))
    per_row = w.nx * w.ppc
    n = nrows * per_row
    threads = threads or min(16, os.cpu_count() or 1)
    if block_rows is None:
        block_rows = max(1, min(nrows, (1 << 21) // max(per_row, 1)))
    x = np.empty(n)
    v = np.empty((w.vdim, n))
    f = np.empty(n)

    def work(r0):
        r1 = min(nrows, r0 + block_rows)
        xs, vs, fs = markers(w, r0, r1)
        a, b = r0 * per_row, r1 * per_row
        x[a:b] = xs
        v[:, a:b] = vs
        f[a:b] = fs

    with ThreadPoolExecutor(threads) as ex:
        list(ex.map(work, range(0, nrows, block_rows)))
    return x, v, f


# ---------------------------------------------------------------------------
# Workloads.  L, dt and the perturbation of the larger cases are not fixed by
# any printed source; the choices below (L = 20*pi so that k_m = 0.1 m, dt =
# 0.1) are this project's and are listed with the other readings.
# ---------------------------------------------------------------------------

def landau_small() -> Workload:
    """Linear Landau damping: k = 0.5, 1% density perturbation, 16,384 markers."""
    return Workload(
        name="landau_1d1v_nx64_nv64_ppc4", vdim=1, nx=64, nv=(64, 1, 1),
        L=4.0 * math.pi, vmin=(-6.0, 0, 0), vmax=(6.0, 0, 0), ppc=4, dt=0.1,
        steps=200, seed=1804, populations=(Population(1.0),),
        mode_numbers=(1,), mode_amplitude=0.01, random_phases=False)


def bump_on_tail(nx: int = 1024, nv: int = 1024, ppc: int = 16, seed: int = 3901,
                 steps: int = 1000, weights: str = "analytic",
                 beam_drift: float = 4.5, beam_density: float = 1e-6) -> Workload:
    """Bump-on-tail: unit core Maxwellian plus a weak beam (drift 4.5, v_th 0.5)."""
    return Workload(
        name=f"bump_on_tail_1d1v_nx{nx}_nv{nv}_ppc{ppc}", vdim=1, nx=nx, nv=(nv, 1, 1),
        L=20.0 * math.pi, vmin=(-8.0, 0, 0), vmax=(8.0, 0, 0), ppc=ppc, dt=0.1,
        steps=steps, seed=seed,
        populations=(Population(1.0), Population(beam_density, (beam_drift, 0, 0), (0.5, 1, 1))),
        mode_numbers=tuple(range(1, 17)), mode_amplitude=1e-4, random_phases=True,
        weights=weights)


def two_stream_3v(nx: int = 512, nv: int = 64, ppc: int = 4, seed: int = 3,
                  steps: int = 100) -> Workload:
    """Two counter-drifting Maxwellians (+-3 along x), isotropic in vy and vz."""
    return Workload(
        name=f"two_stream_1d3v_nx{nx}_nv{nv}^3_ppc{ppc}", vdim=3, nx=nx, nv=(nv, nv, nv),
        L=20.0 * math.pi, vmin=(-8.0, -8.0, -8.0), vmax=(8.0, 8.0, 8.0), ppc=ppc,
        dt=0.1, steps=steps, seed=seed,
        populations=(Population(0.5, (3.0, 0, 0)), Population(0.5, (-3.0, 0, 0))),
        mode_numbers=(1,), mode_amplitude=1e-4, random_phases=False)


def batched_scan(count: int = 64, seed: int = 4000, steps: int = 500, ppc: int = 8,
                 nx_choices: Sequence[int] = (128, 256, 512, 1024),
                 nv_choices: Sequence[int] = (128, 256, 512)) -> list:
    """A parameter scan of bump-on-tail instances of uneven size: instance b
    has nx and nv drawn uniformly from the choices, beam drift uniform in
    [3, 6], beam density log-uniform in [1e-6, 1e-2] (four draws per instance
    from the stream of ``seed``), and markers from seed + b."""
    u = uniforms(seed, 0, 4 * count).reshape(count, 4)
    out = []
    for b in range(count):
        nx = nx_choices[min(int(u[b, 0] * len(nx_choices)), len(nx_choices) - 1)]
        nv = nv_choices[min(int(u[b, 1] * len(nv_choices)), len(nv_choices) - 1)]
        drift = 3.0 + 3.0 * float(u[b, 2])
        dens = 10.0 ** (-6.0 + 4.0 * float(u[b, 3]))
        w = bump_on_tail(nx=nx, nv=nv, ppc=ppc, seed=seed + b, steps=steps, beam_drift=drift, beam_density=dens)
        out.append(w.replace(name=f"scan{b}_nx{nx}_nv{nv}_drift{drift:.3f}_dens{dens:.2e}"))
    return out


def paper_landau(ppc: int = 4, steps: int = 400, seed: int = 1301) -> Workload:
    """The paper's Landau-damping test (Sec. 4.2): box L = 5 pi (longest mode
    k = 0.4), 5% cosine density perturbation of a unit Maxwellian, Nx = 512,
    Nv = 6600 cells on [-5, 5] (a velocity range of ten thermal speeds),
    dt = 0.1, immobile neutralising ions."""
    return Workload(
        name=f"paper_landau_1d1v_nx512_nv6600_ppc{ppc}", vdim=1, nx=512, nv=(6600, 1, 1),
        L=5.0 * math.pi, vmin=(-5.0, 0, 0), vmax=(5.0, 0, 0), ppc=ppc, dt=0.1,
        steps=steps, seed=seed, populations=(Population(1.0),),
        mode_numbers=(1,), mode_amplitude=0.05, random_phases=False)


def langmuir_noise(nx: int = 256, nv: int = 256, ppc: int = 4, modes: int = 16, amplitude: float = 1e-3,
                   steps: int = 2048, seed: int = 1214) -> Workload:
    """A thermal plasma seeded with small density noise in its longest modes
    (k_m = 0.05 m, m = 1..modes, random phases) for the (k, omega) spectrum of
    Langmuir waves (Sec. 4.1); L = 40 pi, v on [-6, 6], dt = 0.1."""
    return Workload(
        name=f"langmuir_1d1v_nx{nx}_nv{nv}_ppc{ppc}", vdim=1, nx=nx, nv=(nv, 1, 1),
        L=40.0 * math.pi, vmin=(-6.0, 0, 0), vmax=(6.0, 0, 0), ppc=ppc, dt=0.1,
        steps=steps, seed=seed, populations=(Population(1.0),),
        mode_numbers=tuple(range(1, modes + 1)), mode_amplitude=amplitude, random_phases=True)


def bernstein(nx: int = 64, nv: int = 24, ppc: int = 2, B: float = 0.5, modes: int = 16,
              amplitude: float = 1e-3, steps: int = 2048, seed: int = 1495) -> Workload:
    """Electron Bernstein waves (Sec. 4.4): 1D-3V electrons gyrating in a
    uniform field along z, perpendicular to x (cyclotron frequency B for q/m =
    -1, plasma frequency 1, thermal speed 1), seeded with small density noise
    in modes k = 0.1 m (m = 1..modes, random phases); L = 20 pi, v on
    [-5, 5]^3, dt = 0.1, immobile ions."""
    return Workload(
        name=f"bernstein_1d3v_nx{nx}_nv{nv}^3_ppc{ppc}", vdim=3, nx=nx, nv=(nv, nv, nv),
        L=20.0 * math.pi, vmin=(-5.0, -5.0, -5.0), vmax=(5.0, 5.0, 5.0), ppc=ppc, dt=0.1,
        steps=steps, seed=seed, populations=(Population(1.0),),
        mode_numbers=tuple(range(1, modes + 1)), mode_amplitude=amplitude, random_phases=True,
        B=(0.0, 0.0, B))


def ion_acoustic(nx: int = 32, nv_e: int = 1024, nv_i: int = 128, ppc: int = 4, mass_ratio: float = 100.0,
                 ti: float = 0.25, amplitude: float = 1e-2, steps: int = 3000, seed: int = 1418):
    """Electrons (T_e = 1) and mobile ions (charge +1, mass ``mass_ratio``,
    temperature ``ti``) carrying the same cosine density perturbation of the
    longest mode (k = 0.5, L = 4 pi), so the start is neutral and the ions'
    response is an ion-acoustic wave; dt = 0.1.  The electron grid resolves
    the slow resonant electrons (v ~ 0.1) and keeps the grid recurrence time
    2 pi / (k dv) beyond the run.  Returns (electrons, ions)."""
    L = 4.0 * math.pi
    vti = math.sqrt(ti / mass_ratio)
    common = dict(vdim=1, nx=nx, L=L, ppc=ppc, dt=0.1, steps=steps,
                  mode_numbers=(1,), mode_amplitude=amplitude, random_phases=False)
    e = Workload(name=f"ion_acoustic_electrons_nx{nx}_nv{nv_e}", nv=(nv_e, 1, 1), vmin=(-6.0, 0, 0),
                 vmax=(6.0, 0, 0), seed=seed, populations=(Population(1.0),), q=-1.0, m=1.0, **common)
    i = Workload(name=f"ion_acoustic_ions_nx{nx}_nv{nv_i}_mr{mass_ratio:g}", nv=(nv_i, 1, 1),
                 vmin=(-14.0 * vti, 0, 0), vmax=(14.0 * vti, 0, 0), seed=seed + 1,
                 populations=(Population(1.0, vth=(vti, 1.0, 1.0)),), q=1.0, m=mass_ratio, **common)
    return e, i


def current_driven(nx: int = 32, nv_e: int = 1024, nv_i: int = 128, ppc: int = 4, mass_ratio: float = 100.0,
                   ti: float = 0.1, drift: float = 1.5, amplitude: float = 1e-3, steps: int = 3000,
                   seed: int = 1457):
    """Current-driven ion-acoustic instability (Sec. 4.3): electrons (T_e = 1)
    drifting by ``drift`` relative to ions (charge +1, mass ``mass_ratio``,
    temperature ``ti``), the centre of mass at rest, both species carrying the
    same small cosine density perturbation of the longest mode (k = 0.5,
    L = 4 pi); dt = 0.1.  Returns (electrons, ions)."""
    L = 4.0 * math.pi
    vti = math.sqrt(ti / mass_ratio)
    ue = drift * mass_ratio / (mass_ratio + 1.0)
    ui = -drift / (mass_ratio + 1.0)
    common = dict(vdim=1, nx=nx, L=L, ppc=ppc, dt=0.1, steps=steps,
                  mode_numbers=(1,), mode_amplitude=amplitude, random_phases=False)
    e = Workload(name=f"cdiai_electrons_nx{nx}_nv{nv_e}", nv=(nv_e, 1, 1), vmin=(ue - 6.5, 0, 0),
                 vmax=(ue + 6.5, 0, 0), seed=seed, populations=(Population(1.0, (ue, 0, 0)),), q=-1.0, m=1.0,
                 **common)
    i = Workload(name=f"cdiai_ions_nx{nx}_nv{nv_i}_mr{mass_ratio:g}", nv=(nv_i, 1, 1),
                 vmin=(ui - 14.0 * vti, 0, 0), vmax=(ui + 14.0 * vti, 0, 0), seed=seed + 1,
                 populations=(Population(1.0, (ui, 0, 0), (vti, 1.0, 1.0)),), q=1.0, m=mass_ratio, **common)
    return e, i


def adjoint_case() -> Workload:
    return bump_on_tail(nx=1024, nv=512, ppc=8, seed=5, steps=500)


WORKLOADS = {
    "landau": landau_small,
    "bump_on_tail": bump_on_tail,
    "two_stream_3v": two_stream_3v,
    "adjoint": adjoint_case,
    "paper_landau": paper_landau,
    "langmuir": langmuir_noise,
    "bernstein": bernstein,
}
