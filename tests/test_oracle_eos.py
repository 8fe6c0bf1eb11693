"""Pins of the constant-w kernels (oracle/eos.py), the kernel-table variant
for other equations of state (Sec. II equations, Sec. IV time integrals).

* w = 1/3 reduces to the paper: the numerically evaluated I_s^w, I_c^w equal
  the closed forms of Eq. kernels on every cell of the default strip,
  including cells within 1e-4 of the resonance u + v = sqrt(3) where I_c
  diverges logarithmically; the transfer function and the source factor
  equal the radiation-era ones of the oracle's kernels module.
* Other w: the building blocks solve the equations they come from
  (Eq. scalar with c_s^2 = w, the homogeneous wave equation of Sec. II,
  Abel's identity for the Wronskian, D = T + H^-1 dT/deta), and the kernels
  agree with a second, independent evaluation of the same time integrals
  (exp(-eps t) damping on the real line, Simpson, eps -> 0 extrapolation) at
  the P5 points away from the resonance sqrt(w)(u + v) = 1.
A sign error in a Hankel term, a wrong weight power, a dropped source factor
or a wrong ray direction fails one of these.
"""
import math

import numpy as np
import pytest

from oracle import decomposition, eos, kernels

POINTS = [(0.8, 0.7), (1.2, 0.9), (0.6, 0.5), (1.5, 1.3), (2.5, 2.0)]


def test_w_one_third_reproduces_eq_kernels_on_the_strip():
    e = decomposition.grid_edges(200, 1e-3, 15.0, 1.0, 0.5, 10.0)
    c = 0.5 * (e[1:] + e[:-1])
    Is, Ic = eos.kernel_matrices(c, 1.0 / 3.0)
    U, V = np.meshgrid(c, c, indexing="ij")
    strip = (np.abs(U - V) <= 1.0) & (U + V >= 1.0)
    near = strip & (np.abs(U + V - math.sqrt(3.0)) < 1e-4)
    assert near.any()
    for got, ref in ((Is, kernels.I_s(U, V)), (Ic, kernels.I_c(U, V))):
        scale = np.abs(ref[strip]).max()
        err = np.abs(got - ref)[strip]
        assert err.max() <= 1e-8 * scale
        big = strip & (np.abs(ref) > 1e-2 * scale)
        assert np.max(np.abs(got - ref)[big] / np.abs(ref[big])) <= 1e-7


def test_w_one_third_building_blocks():
    x = np.linspace(1e-3, 40.0, 2001)
    np.testing.assert_allclose(eos.transfer(x, 1.0 / 3.0), kernels.transfer(x * math.sqrt(3.0)), atol=1e-13)
    np.testing.assert_allclose(eos.transfer_D(x, 1.0 / 3.0), kernels.transfer_plus(x * math.sqrt(3.0)), atol=1e-12)
    b, nu, mu, c_src, r = eos.params(1.0 / 3.0)
    assert (b, nu, mu, c_src) == pytest.approx((0.0, 1.5, 0.5, 0.5), abs=1e-15)
    assert r == pytest.approx(1.0, abs=1e-15)
    t = np.linspace(0.5, 30.0, 300)
    y1, y2 = eos.y_solutions(t, 1.0 / 3.0)
    np.testing.assert_allclose(y1, np.cos(t) / t, atol=1e-14)
    np.testing.assert_allclose(y2, np.sin(t) / t, atol=1e-14)


@pytest.mark.parametrize("w", [0.1, 0.2, 0.6, 0.9])
def test_building_blocks_solve_their_equations(w):
    b, nu, mu, c_src, r = eos.params(w)
    h = 1e-3
    # Eq. scalar with c_s^2 = w and H = (1 + b)/eta, at k = 1:
    # T'' + 3 H (1 + w) T' + (2 H' + (1 + 3w) H^2 + w) T = 0, T(0) = 1, T'(0) = 0
    eta = np.linspace(0.2, 40.0, 600)
    T = lambda e: eos.transfer(math.sqrt(w) * e, w)
    d1 = (T(eta + h) - T(eta - h)) / (2 * h)
    d2 = (T(eta + h) - 2 * T(eta) + T(eta - h)) / (h * h)
    H = (1.0 + b) / eta
    dH = -(1.0 + b) / eta ** 2
    resid = d2 + 3.0 * H * (1.0 + w) * d1 + (2.0 * dH + (1.0 + 3.0 * w) * H ** 2 + w) * T(eta)
    assert np.max(np.abs(resid)) < 2e-5
    assert abs(float(T(np.array([1e-6]))[0]) - 1.0) < 1e-9
    assert abs(float((T(np.array([2e-6])) - T(np.array([1e-6])))[0])) < 1e-9
    # D = T + H^-1 dT/deta
    np.testing.assert_allclose(eos.transfer_D(math.sqrt(w) * eta, w), T(eta) + d1 / H, atol=1e-6)
    # homogeneous wave equation y'' + 2 H y' + y = 0 (k = 1, t = eta) and the Wronskian
    t = np.linspace(1.0, 40.0, 600)      # away from t = 0, where y1 ~ t^-(1+2b) defeats the finite difference
    for k in (0, 1):
        y = lambda s: eos.y_solutions(s, w)[k]
        r2 = ((y(t + h) - 2 * y(t) + y(t - h)) / (h * h) + 2.0 * (1.0 + b) / t * (y(t + h) - y(t - h)) / (2 * h)
              + y(t))
        assert np.max(np.abs(r2)) < 1e-4 * max(1.0, float(np.max(np.abs(y(t)))))
    y1, y2 = eos.y_solutions(t, w)
    y1d = (eos.y_solutions(t + h, w)[0] - eos.y_solutions(t - h, w)[0]) / (2 * h)
    y2d = (eos.y_solutions(t + h, w)[1] - eos.y_solutions(t - h, w)[1]) / (2 * h)
    np.testing.assert_allclose(y1 * y2d - y1d * y2, t ** (-2.0 * (1.0 + b)), rtol=1e-5)


@pytest.mark.slow
@pytest.mark.parametrize("w", [0.2, 0.6])
def test_kernels_agree_with_damped_real_line_integrals(w):
    c = np.array(sorted({x for p in POINTS for x in p}))
    Is, Ic = eos.kernel_matrices(c, w)
    idx = {x: i for i, x in enumerate(c)}
    checked = 0
    for u, v in POINTS:
        if abs(math.sqrt(w) * (u + v) - 1.0) < 0.1:
            continue                       # the damped route is inaccurate next to the resonance
        for which, M in (("s", Is), ("c", Ic)):
            num = eos.time_integral_damped(u, v, w, which)
            got = M[idx[u], idx[v]]
            assert abs(got - num) <= 1e-3 * max(abs(num), 1.0), (w, u, v, which, got, num)
            checked += 1
    assert checked >= 6
