"""Pins of the closed-form kernels (Eq. kernels) and their physics inputs.

P5: the closed forms equal the defining time integrals
    I_{s,c}(u,v) = int_0^inf dt t {sin,cos}(t) f(t,u,v)
evaluated by independent quadrature (damped, Richardson-extrapolated), at
points on both sides of the resonance u + v = sqrt(3).  A wrong sign, a
dropped term or a wrong power in Eq. kernels fails here.
Also pinned: the transfer function's textbook limits (T(0) = 1, the w = 1/3
solution of the potential equation), symmetry I(u,v) = I(v,u), the Theta
cut of I_s at u + v = sqrt(3), and the logarithmic divergence of I_c there.
"""
import math

import numpy as np
import pytest

from oracle import kernels

POINTS = [(0.8, 0.7), (1.2, 0.9), (0.6, 0.5), (1.5, 1.3), (2.5, 2.0)]


@pytest.mark.parametrize("u,v", POINTS)
def test_closed_forms_equal_time_integrals(u, v):
    for which, f in (("s", kernels.I_s), ("c", kernels.I_c)):
        num = kernels.time_integral(u, v, which)
        ref = float(f(u, v))
        scale = max(abs(ref), 0.1)
        assert abs(num - ref) <= 1e-3 * scale, (which, u, v, num, ref)


def test_kernel_symmetry_and_theta_cut():
    rng = np.random.default_rng(1)
    u = rng.uniform(0.05, 5, 200)
    v = rng.uniform(0.05, 5, 200)
    np.testing.assert_allclose(kernels.I_s(u, v), kernels.I_s(v, u), rtol=1e-14)
    np.testing.assert_allclose(kernels.I_c(u, v), kernels.I_c(v, u), rtol=1e-14)
    r3 = math.sqrt(3.0)
    assert kernels.I_s(0.8, r3 - 0.8 - 1e-9) == 0.0
    assert kernels.I_s(0.8, r3 - 0.8 + 1e-9) > 0.0
    # I_c diverges logarithmically at the resonance u + v = sqrt(3)
    a = abs(float(kernels.I_c(0.8, r3 - 0.8 + 1e-4)))
    b = abs(float(kernels.I_c(0.8, r3 - 0.8 + 1e-8)))
    assert b > a * 1.5


def test_transfer_function_solves_potential_equation():
    """T(x) = 3 j1(y)/y, y = x/sqrt3, solves Phi'' + (4/eta) Phi' + k^2/3 Phi = 0
    in radiation domination (c_s^2 = 1/3, H = 1/eta), with T(0) = 1, T'(0) = 0."""
    x = np.linspace(0.05, 30.0, 4001)
    h = 1e-3
    T = kernels.transfer
    d1 = (T(x + h) - T(x - h)) / (2 * h)
    d2 = (T(x + h) - 2 * T(x) + T(x - h)) / (h * h)
    resid = d2 + 4.0 / x * d1 + T(x) / 3.0
    assert np.max(np.abs(resid)) < 5e-6
    assert abs(float(T(np.array([1e-8]))[0]) - 1.0) < 1e-12
    # T + x T' against a finite difference of x T(x)
    g = (x + h) * T(x + h) - (x - h) * T(x - h)
    np.testing.assert_allclose(kernels.transfer_plus(x), g / (2 * h), atol=1e-6)
