"""Parity measures shared by the GPU tests.

f, D and rho are compared normwise (max|gpu - oracle| / max|oracle|) and f
also cell by cell (cell_rel) wherever the oracle's weight sum D is at least
D_FLOOR, a tenth of one marker's full weight: there f is a normalised average
of marker weights, so its relative error means something however small f
is (the low-f cells Eq. (reconstruction) protects).


The field is checked at its own scale, max|E|, in two parts (Sec. 2,
Eq. (poissonk), Eq. (kappasoftening)):

* the GPU's solve of its OWN charge density against the oracle's solve of
  that same rho, at 1e-12 of max|E| (both sides solve in FP64, so this bound
  holds for every storage form);
* the field the GPU reached against the oracle's, bounded by the charge error
  actually measured, propagated through the Poisson map:
      max|E_g - E_o| <= G max|rho_g - rho_o| + 1e-12 max|E_o|,
  with G the exact infinity-norm gain of the oracle's map (the map is a
  convolution, so G is the l1 norm of its response to a unit impulse).

The field energy W = sum E^2 dx / (2 c_P) (Sec. 3.4) is held to the algebraic
bound that follows from the measured fields: W_g - W_o = sum (E_g - E_o)(E_g +
E_o) dx / (2 c_P), plus 1e-12 of W for the GPU's own reduction.

TOL_SOLVE is the per-step FP64 bound; the oracle and the GPU both remove the
mean of rho before their transforms (the k = 0 mode is dropped), which leaves
both at ~1e-15 of max|E| on the charge densities of these runs.
"""
from functools import lru_cache

import numpy as np

import oracle

TOL_SOLVE = 1e-12
D_FLOOR = 0.1


def nrel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    s = np.max(np.abs(b))
    return float(np.max(np.abs(a - b)) / s) if s > 0 else float(np.max(np.abs(a - b)))


def cell_rel(f_g, f_o, D_o, floor=D_FLOOR):
    """Largest |f_g - f_o| / |f_o| over the cells with D_o >= floor."""
    f_g = np.asarray(f_g, dtype=np.float64).reshape(-1)
    f_o = np.asarray(f_o, dtype=np.float64).reshape(-1)
    D_o = np.asarray(D_o, dtype=np.float64).reshape(-1)
    m = (D_o >= floor) & (f_o != 0)
    if not np.any(m):
        return 0.0
    return float(np.max(np.abs(f_g[m] - f_o[m]) / np.abs(f_o[m])))


@lru_cache(maxsize=None)
def poisson_gain(nx, L, c_p):
    """Infinity-norm gain of the oracle's Poisson map on an nx grid."""
    e0 = np.zeros(nx)
    e0[0] = 1.0
    g, _ = oracle.poisson(nx, L, c_p, e0)
    return float(np.sum(np.abs(g)))


def check_field(w, rho_g, E_g, rho_o, E_o, W_g=None, label=""):
    """Assert the two field bounds (and W's, if W_g is given); returns the
    measured errors relative to max|E_o| for reporting."""
    rho_g = np.asarray(rho_g, dtype=np.float64)
    E_g = np.asarray(E_g, dtype=np.float64)
    rho_o = np.asarray(rho_o, dtype=np.float64)
    E_o = np.asarray(E_o, dtype=np.float64)
    Emax = max(float(np.max(np.abs(E_o))), 1e-300)
    # 1. the GPU's solve of its own rho, against the oracle's solve of it
    E_gsolve, _ = oracle.poisson(w.nx, w.L, w.c_p, rho_g)
    solve_err = float(np.max(np.abs(E_g - E_gsolve))) / max(float(np.max(np.abs(E_gsolve))), 1e-300)
    assert solve_err <= TOL_SOLVE, f"{label}: solve of the GPU's rho off by {solve_err:.3e} of max|E|"
    # 2. the field reached, against the oracle's, within the propagated charge error
    G = poisson_gain(w.nx, w.L, w.c_p)
    drho = float(np.max(np.abs(rho_g - rho_o)))
    dE = float(np.max(np.abs(E_g - E_o)))
    bound = G * drho * (1.0 + 1e-9) + TOL_SOLVE * Emax
    assert dE <= bound, f"{label}: max|dE| {dE:.3e} above G max|drho| + 1e-12 max|E| = {bound:.3e}"
    out = {"E_solve": solve_err, "E": dE / Emax, "E_bound": bound / Emax}
    if W_g is not None:
        dx = w.L / w.nx
        W_o = oracle.field_energy(w.nx, w.L, w.c_p, E_o)
        wb = float(np.sum(np.abs(E_g + E_o) * np.abs(E_g - E_o))) * dx / (2 * w.c_p) * (1.0 + 1e-9)
        assert abs(float(W_g) - W_o) <= wb + TOL_SOLVE * W_o, \
            f"{label}: |W_g - W_o| {abs(float(W_g) - W_o):.3e} above {wb + TOL_SOLVE * W_o:.3e}"
        out["W"] = abs(float(W_g) - W_o) / W_o if W_o > 0 else abs(float(W_g) - W_o)
    return out
