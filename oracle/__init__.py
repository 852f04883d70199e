"""Python entry to the plain FP64 CPU oracle (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It compiles ``avl_oracle.c`` with gcc
(``-O2 -ffp-contract=off``, single thread) into ``oracle/_build`` and calls it
through ctypes.  Nothing here touches the GPU library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "avl_oracle.c")
_BUILD = os.path.join(_HERE, "_build")
_LIB = os.path.join(_BUILD, "liboracle.so")
_lock = threading.Lock()
_lib = None


class OrcGrid(ctypes.Structure):
    _fields_ = [
        ("vdim", ctypes.c_int32), ("nx", ctypes.c_int32), ("nv", ctypes.c_int32 * 3),
        ("pad_", ctypes.c_int32),
        ("L", ctypes.c_double), ("vmin", ctypes.c_double * 3), ("vmax", ctypes.c_double * 3),
        ("dt", ctypes.c_double), ("q", ctypes.c_double), ("m", ctypes.c_double),
        ("cp", ctypes.c_double), ("B", ctypes.c_double * 3),
    ]


def build(force: bool = False) -> str:
    """Compile the oracle (always when ``force``)."""
    os.makedirs(_BUILD, exist_ok=True)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11",
                               "-Wall", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB)
            P = ctypes.POINTER
            d = ctypes.c_double
            pd = P(d)
            g = P(OrcGrid)
            L = ctypes.c_long
            lib.orc_reconstruct.argtypes = [g, L, pd, pd, pd, pd, pd, pd]
            lib.orc_reconstruct.restype = ctypes.c_int
            lib.orc_deposit_naive.argtypes = [g, L, pd, pd, pd, pd]
            lib.orc_deposit_naive.restype = ctypes.c_int
            lib.orc_moments.argtypes = [g, pd, pd, pd, pd]
            lib.orc_moments.restype = None
            lib.orc_poisson.argtypes = [ctypes.c_int, d, d, pd, pd, pd]
            lib.orc_poisson.restype = ctypes.c_int
            lib.orc_field_energy.argtypes = [ctypes.c_int, d, d, pd]
            lib.orc_field_energy.restype = d
            lib.orc_energy.argtypes = [g, pd, pd, pd, pd]
            lib.orc_energy.restype = None
            lib.orc_residual.argtypes = [ctypes.c_int, d, d, pd, pd, pd]
            lib.orc_residual.restype = None
            lib.orc_push.argtypes = [g, L, pd, pd, pd, d]
            lib.orc_push.restype = None
            lib.orc_run.argtypes = [g, L, pd, pd, pd, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                    pd, pd, pd, pd, pd]
            lib.orc_run.restype = ctypes.c_int
            _lib = lib
    return _lib


def _p(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class Grid:
    """Grid and species constants, mirrored from an ``inputs.Workload`` or given directly."""

    def __init__(self, vdim, nx, nv, L, vmin, vmax, dt=0.1, q=-1.0, m=1.0, cp=1.0, B=(0.0, 0.0, 0.0)):
        nv = tuple(nv) + (1,) * (3 - len(tuple(nv)))
        vmin = tuple(vmin) + (0.0,) * (3 - len(tuple(vmin)))
        vmax = tuple(vmax) + (0.0,) * (3 - len(tuple(vmax)))
        self.vdim, self.nx, self.nv, self.L = int(vdim), int(nx), nv, float(L)
        self.vmin, self.vmax, self.dt, self.q, self.m, self.cp = vmin, vmax, float(dt), float(q), float(m), float(cp)
        self.B = tuple(float(b) for b in B)
        self.c = OrcGrid(self.vdim, self.nx, (ctypes.c_int32 * 3)(*nv), 0, self.L,
                         (ctypes.c_double * 3)(*vmin), (ctypes.c_double * 3)(*vmax),
                         self.dt, self.q, self.m, self.cp, (ctypes.c_double * 3)(*self.B))

    @classmethod
    def from_workload(cls, w):
        return cls(w.vdim, w.nx, w.nv, w.L, w.vmin, w.vmax, w.dt, w.q, w.m, w.c_p, getattr(w, "B", (0.0, 0.0, 0.0)))

    @property
    def n_cells(self):
        c = self.nx
        for d in range(self.vdim):
            c *= self.nv[d]
        return c

    @property
    def grid_shape(self):
        """Shape of phase-space arrays, slowest index first: (nvz, nvy, nvx, nx) or (nv, nx)."""
        return tuple(self.nv[d] for d in reversed(range(self.vdim))) + (self.nx,)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def reconstruct(grid: Grid, x, v, f):
    """Returns (N, D, f_grid) of Eq. (reconstruction), each shaped ``grid.grid_shape``."""
    lib = _load()
    x, f = _f64(x), _f64(f)
    v = _f64(np.reshape(v, (grid.vdim, -1)))
    n = x.size
    N = np.empty(grid.n_cells)
    D = np.empty(grid.n_cells)
    fg = np.empty(grid.n_cells)
    rc = lib.orc_reconstruct(ctypes.byref(grid.c), n, _p(x), _p(v), _p(f), _p(N), _p(D), _p(fg))
    assert rc == 0
    s = grid.grid_shape
    return N.reshape(s), D.reshape(s), fg.reshape(s)


def deposit_naive(grid: Grid, x, v, f):
    lib = _load()
    x, f = _f64(x), _f64(f)
    v = _f64(np.reshape(v, (grid.vdim, -1)))
    out = np.empty(grid.n_cells)
    lib.orc_deposit_naive(ctypes.byref(grid.c), x.size, _p(x), _p(v), _p(f), _p(out))
    return out.reshape(grid.grid_shape)


def moments(grid: Grid, fg):
    """Returns (rho, jx, m2) on the nx cell centres."""
    lib = _load()
    fg = _f64(fg).reshape(-1)
    rho, jx, m2 = np.empty(grid.nx), np.empty(grid.nx), np.empty(grid.nx)
    lib.orc_moments(ctypes.byref(grid.c), _p(fg), _p(rho), _p(jx), _p(m2))
    return rho, jx, m2


def poisson(nx, L, cp, rho):
    """Returns (E, mode-1 amplitude of E)."""
    lib = _load()
    rho = _f64(rho)
    E = np.empty(nx)
    m1 = ctypes.c_double(0.0)
    rc = lib.orc_poisson(int(nx), float(L), float(cp), _p(rho), _p(E), ctypes.byref(m1))
    assert rc == 0
    return E, m1.value


def field_energy(nx, L, cp, E):
    return _load().orc_field_energy(int(nx), float(L), float(cp), _p(_f64(E)))


def energy(grid: Grid, fg):
    lib = _load()
    fg = _f64(fg).reshape(-1)
    a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    lib.orc_energy(ctypes.byref(grid.c), _p(fg), ctypes.byref(a), ctypes.byref(b), ctypes.byref(c))
    return a.value, b.value, c.value


def residual(nx, L, cp, rho, E):
    """Residual charge (rho - mean rho) - centred dE/dx / cp on the nx cells."""
    out = np.empty(int(nx))
    _load().orc_residual(int(nx), float(L), float(cp), _p(_f64(rho)), _p(_f64(E)), _p(out))
    return out


def push(grid: Grid, x, v, E, kick=1.0):
    """Gather + kick + drift + wrap; returns new (x, v) copies."""
    lib = _load()
    x = _f64(x).copy()
    v = _f64(np.reshape(v, (grid.vdim, -1))).copy()
    lib.orc_push(ctypes.byref(grid.c), x.size, _p(x), _p(v), _p(_f64(E)), float(kick))
    return x, v


def run(grid: Grid, x, v, f, nsteps, first_kick_half=False, E=None):
    """Initial solve (unless E is given) then ``nsteps`` steps.

    Returns dict with x, v (final), E, diag[nsteps, 2] = (W, |E_hat_1|), f, D, rho.
    """
    lib = _load()
    x = _f64(x).copy()
    v = _f64(np.reshape(v, (grid.vdim, -1))).copy()
    f = _f64(f)
    have = E is not None
    E = _f64(E).copy() if have else np.zeros(grid.nx)
    diag = np.zeros((max(nsteps, 1), 2))
    fg = np.empty(grid.n_cells)
    D = np.empty(grid.n_cells)
    rho = np.empty(grid.nx)
    rc = lib.orc_run(ctypes.byref(grid.c), x.size, _p(x), _p(v), _p(f), int(nsteps),
                     int(bool(first_kick_half)), int(have), _p(E), _p(diag), _p(fg), _p(D), _p(rho))
    assert rc == 0
    s = grid.grid_shape
    return {"x": x, "v": v, "E": E, "diag": diag[:nsteps], "f": fg.reshape(s),
            "D": D.reshape(s), "rho": rho}
