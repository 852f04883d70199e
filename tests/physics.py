"""Test-side analysis helpers, independent of both the oracle and the GPU path.

* ``cic_overlap_bruteforce``: the cloud-in-cell weight computed as the literal
  area of overlap between a marker's cell-sized cloud and each grid cell (the
  picture of Sec. 2, Fig. "interpolation"), with exact rational arithmetic and
  periodic images in x.  A different derivation from the closed-form corner
  weights the oracle uses.
* ``landau_root``: the exact linear Landau root of a unit Maxwellian from the
  plasma dispersion function (Z(zeta) = i sqrt(pi) w(zeta), Faddeeva w from
  scipy), which the paper does not print.
* ``damping_rate``: least-squares slope of log peak amplitudes, the fitting
  procedure of Sec. 4.2 (peaks of the mode amplitude, fit over a time window).
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np


def _overlap(lo1, hi1, lo2, hi2):
    return max(Fraction(0), min(hi1, hi2) - max(lo1, lo2))


def cic_overlap_bruteforce(nx, L, nvs, vmins, vmaxs, markers):
    """Exact N, D arrays (Fractions) for markers [(x, (v...), f)] on a tiny grid.

    Returns dicts keyed by (i, j0[, j1, j2]) -> (N, D).
    """
    L = Fraction(L)
    dx = L / nx
    dvs = [(Fraction(vmaxs[d]) - Fraction(vmins[d])) / nvs[d] for d in range(len(nvs))]
    N, D = {}, {}
    import itertools
    for (x, vs, f) in markers:
        x = Fraction(x)
        f = Fraction(f)
        vs = [Fraction(v) for v in vs]
        for idx in itertools.product(range(nx), *[range(n) for n in nvs]):
            i = idx[0]
            ox = Fraction(0)
            for p in (-1, 0, 1):
                ox += _overlap(x - dx / 2 + p * L, x + dx / 2 + p * L, i * dx, (i + 1) * dx)
            w = ox / dx
            for d, j in enumerate(idx[1:]):
                lo = Fraction(vmins[d]) + j * dvs[d]
                w *= _overlap(vs[d] - dvs[d] / 2, vs[d] + dvs[d] / 2, lo, lo + dvs[d]) / dvs[d]
            if w:
                N[idx] = N.get(idx, Fraction(0)) + w * f
                D[idx] = D.get(idx, Fraction(0)) + w
    return N, D


def landau_root(k: float, guess=None) -> complex:
    """Complex frequency of the least-damped Langmuir mode of a unit Maxwellian
    (v_th = 1, omega_p = 1): 1 + (1 + zeta Z(zeta)) / k^2 = 0, zeta = omega/(sqrt2 k)."""
    from scipy.special import wofz

    def eps(w):
        z = w / (math.sqrt(2.0) * k)
        Z = 1j * math.sqrt(math.pi) * wofz(z)
        return 1.0 + (1.0 + z * Z) / (k * k)

    w = complex(guess) if guess is not None else complex(math.sqrt(1 + 3 * k * k), -0.1)
    for _ in range(100):
        h = 1e-7
        d = (eps(w + h) - eps(w - h)) / (2 * h)
        step = eps(w) / d
        w -= step
        if abs(step) < 1e-14:
            break
    return w


def peaks(amp, dt, half_window=1.0):
    """Local maxima of amp (sampled at t = (n+1) dt) that are the largest value
    within +-half_window, refined by a parabola through log amplitudes."""
    amp = np.asarray(amp)
    t = (np.arange(len(amp)) + 1) * dt
    h = max(1, int(round(half_window / dt)))
    out = []
    for n in range(1, len(amp) - 1):
        a, b = max(0, n - h), min(len(amp), n + h + 1)
        if amp[n] == amp[a:b].max() and amp[n] > 0:
            y0, y1, y2 = np.log(amp[n - 1:n + 2])
            den = y0 - 2 * y1 + y2
            dl = 0.5 * (y0 - y2) / den if den != 0 else 0.0
            out.append((t[n] + dl * dt, y1 - 0.25 * (y0 - y2) * dl))
    return np.array(out)


def damping_rate(amp, dt, t_lo=1.5, t_hi=20.0, t_freq=15.0, half_window=1.0):
    """(gamma, omega) from peaks of |E_1|: slope of log peaks over [t_lo, t_hi],
    and pi / (regression slope of peak time on peak index) over [t_lo, t_freq]
    (|E_1| peaks twice per wave period; late peaks sit near the noise floor)."""
    pk = peaks(amp, dt, half_window)
    sel = (pk[:, 0] >= t_lo) & (pk[:, 0] <= t_hi)
    A = np.vstack([np.ones(sel.sum()), pk[sel, 0]]).T
    gamma = np.linalg.lstsq(A, pk[sel, 1], rcond=None)[0][1]
    tf = pk[(pk[:, 0] >= t_lo) & (pk[:, 0] <= t_freq), 0]
    spacing = np.polyfit(np.arange(tf.size), tf, 1)[0]
    return gamma, math.pi / spacing


def bernstein_roots(k: float, wc: float, wp: float = 1.0, vt: float = 1.0, bands: int = 4, nmax: int = 60):
    """Frequencies of electrostatic electron Bernstein waves (k perpendicular
    to B, Maxwellian electrons of thermal speed vt, immobile ions), one in each
    band (n wc, (n+1) wc) for n = 1..bands: the roots of
    1 = (wp/wc)^2 (e^-lam / lam) sum_{n>=1} 2 n^2 I_n(lam) / ((w/wc)^2 - n^2),
    lam = (k vt / wc)^2, found by bisection (the right side falls from +inf
    to -inf across each band)."""
    from scipy.special import ive
    lam = (k * vt / wc) ** 2
    ns = np.arange(1, nmax + 1)
    coef = 2.0 * ns ** 2 * ive(ns, lam) / lam * (wp / wc) ** 2

    def F(w):
        return 1.0 - float(np.sum(coef / ((w / wc) ** 2 - ns ** 2)))

    out = []
    for n in range(1, bands + 1):
        lo, hi = n * wc * (1 + 1e-12), (n + 1) * wc * (1 - 1e-12)
        flo, fhi = F(lo), F(hi)
        if not (flo < 0 < fhi):
            out.append(float("nan"))
            continue
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if F(mid) < 0:
                lo = mid
            else:
                hi = mid
        out.append(0.5 * (lo + hi))
    return out


def multi_species_root(k: float, species, guess: complex) -> complex:
    """Complex frequency of an electrostatic mode of several drifting
    Maxwellian species (normalised units, c_p = 1): the root near ``guess`` of
    1 + sum_s n_s q_s^2 / (T_s k^2) (1 + zeta_s Z(zeta_s)) = 0 with
    zeta_s = (omega - k u_s) / (sqrt(2) k v_s), v_s = sqrt(T_s / m_s);
    ``species`` holds (n, q, m, T, u) per species."""
    from scipy.special import wofz

    def eps(w):
        tot = 1.0 + 0j
        for n, q, m, T, u in species:
            vs = math.sqrt(T / m)
            z = (w - k * u) / (math.sqrt(2.0) * k * vs)
            Z = 1j * math.sqrt(math.pi) * wofz(z)
            tot += n * q * q / (T * k * k) * (1.0 + z * Z)
        return tot

    w = complex(guess)
    for _ in range(200):
        h = 1e-8 * max(1.0, abs(w))
        d = (eps(w + h) - eps(w - h)) / (2 * h)
        step = eps(w) / d
        w -= step
        if abs(step) < 1e-14 * max(1.0, abs(w)):
            break
    return w
