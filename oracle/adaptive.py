"""Per-target box of the paper's measurement protocol (Sec. VI, lattice setup).

For each target k the box side follows from the Nyquist frequency,
L = pi N / k_max, with k_max = 3 max(k, k_bar), where k_bar is the
wavenumber below which a fraction 1 - eps of the spectrum's power (in
d log k) lies; eps = 0.1 in the paper.  The field is generated anew in that
box (same seed) and Omega is measured in the thin shell k +- pi/L.

k_bar is found here by adaptive quadrature of Delta^2 over log k and root
bracketing: no closed form of the log-normal is used.

Test infrastructure only: nothing on the product path imports this.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate, optimize

from . import decomposition, field, spectrum


def power_fraction_below(k: float, spec) -> float:
    """int_0^k dlog q Delta^2(q) / int_0^inf dlog q Delta^2(q)."""
    f = lambda t: float(field.lognormal_delta2(math.exp(t), spec.A, spec.sigma, spec.k_star))
    c = math.log(spec.k_star)
    w = 40.0 * spec.sigma
    tot = integrate.quad(f, c - w, c + w, points=[c], limit=400, epsabs=0, epsrel=1e-13)[0]
    lk = math.log(k)
    if lk <= c - w:
        return 0.0
    part = integrate.quad(f, c - w, min(lk, c + w), limit=400, epsabs=0, epsrel=1e-13)[0]
    return part / tot


def k_bar(spec, eps: float) -> float:
    lo, hi = spec.k_star * math.exp(-30 * spec.sigma), spec.k_star * math.exp(30 * spec.sigma)
    return optimize.brentq(lambda k: power_fraction_below(k, spec) - (1.0 - eps), lo, hi, xtol=1e-15,
                           rtol=4 * np.finfo(float).eps, maxiter=500)


def box_for_target(N: int, k: float, spec, eps: float) -> float:
    return math.pi * N / (3.0 * max(k, k_bar(spec, eps)))


def omega_adaptive(N: int, seed: int, spec, ngmap, targets, eps: float = 0.1, tabs=None):
    """(Omega, N_b, L) per target."""
    tabs = tabs or decomposition.tables()
    out = []
    for k in targets:
        L = box_for_target(N, float(k), spec, eps)
        ph = field.phi_hat(N, L, seed, spec, ngmap)
        om, nb = spectrum.omega_target(ph, tabs[0], tabs[1], float(k), k - math.pi / L, k + math.pi / L, L)
        out.append((om, nb, L))
    return out
