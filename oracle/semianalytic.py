"""Semi-analytic Omega_GW for Gaussian curvature perturbations (Eq. semi_anal).

    Omega^(RD,Gauss)(k) = int_0^1 dq int_1^inf ds T(q, s) Delta^2(k (s+q)/2) Delta^2(k (s-q)/2)

    T(q, s) = 12 (q^2+s^2-6)^4 / (s^2-q^2)^8 (q^2-1)^2 (s^2-1)^2
              * [ (ln|(3-q^2)/(3-s^2)| + 2(s^2-q^2)/(q^2+s^2-6))^2 + pi^2 Theta(s - sqrt3) ]

The s integral is split at the logarithmic singularity s = sqrt(3) and cut
where the log-normal factors have decayed below double precision.  Above
sqrt(3) it can be split further into `pieces` geometric intervals, which a
narrow (sigma = 0.1) or wide (sigma = 1) peak needs for the adaptive
quadrature to find all of its weight; the result must not depend on it.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate

from .field import lognormal_delta2

SQRT3 = math.sqrt(3.0)


def T_kernel(q, s):
    q = np.asarray(q, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64)
    q2, s2 = q * q, s * s
    with np.errstate(divide="ignore", invalid="ignore"):
        lg = np.log(np.abs((3.0 - q2) / (3.0 - s2)))
        br = (lg + 2.0 * (s2 - q2) / (q2 + s2 - 6.0)) ** 2 + math.pi ** 2 * (s > SQRT3)
        return 12.0 * (q2 + s2 - 6.0) ** 4 / (s2 - q2) ** 8 * (q2 - 1.0) ** 2 * (s2 - 1.0) ** 2 * br


def omega_gauss(k: float, A: float, sigma: float, k_star: float, epsrel: float = 1e-8, pieces: int = 1) -> float:
    def f(s, q):
        return float(T_kernel(q, s) * lognormal_delta2(k * (s + q) / 2.0, A, sigma, k_star)
                     * lognormal_delta2(k * (s - q) / 2.0, A, sigma, k_star))
    # beyond s_max both Delta^2 factors are below exp(-40) of their peak
    s_max = max(2.0 * k_star / k * math.exp(9.0 * sigma) + 1.0, SQRT3 + 1.0)
    cuts = [SQRT3] + list(np.geomspace(SQRT3, s_max, pieces + 1)[1:])
    total = 0.0
    for a, b in [(1.0, SQRT3)] + list(zip(cuts[:-1], cuts[1:])):
        val, _ = integrate.dblquad(f, 0.0, 1.0, lambda q: a, lambda q: b,
                                   epsabs=0.0, epsrel=epsrel)
        total += val
    return total
