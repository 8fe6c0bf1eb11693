"""Pins of the Gaussian realisation and the maps (Sec. VI; P11, P12 statistics).

* the measured shell power of zeta_g matches the input P(k) = 2 pi^2 Delta^2/k^3
  within cosmic variance (chi^2 over shells), so a wrong dV, V or sqrt fails;
* the sample variance of zeta_g matches (1/V) sum_n P(k_n), the lattice
  version of int Delta^2 dln k (which the log-normal makes equal to A);
* Phi_hat = (2/3) dV DFT(zeta) and is Hermitian on the self-conjugate planes;
* local map with the sample mean subtracted has the stated moments; the
  exponential-tail map is clipped where 1 - beta zeta_g falls below the clip.
"""
import math

import numpy as np
import pytest
from scipy import integrate

import workloads as W
from oracle import field, lattice


def test_lognormal_integrates_to_amplitude():
    A, s, ks = 1e-2, 0.5, 20.0
    val, _ = integrate.quad(lambda lk: float(field.lognormal_delta2(math.exp(lk), A, s, ks)),
                            math.log(ks) - 12 * s, math.log(ks) + 12 * s, epsrel=1e-12)
    assert val == pytest.approx(A, rel=1e-10)
    assert float(field.power_spectrum(ks, A, s, ks)) == pytest.approx(
        2 * math.pi ** 2 * A / math.sqrt(2 * math.pi * s * s) / ks ** 3, rel=1e-14)


def test_shell_power_matches_input():
    N, L = 48, 2 * math.pi
    spec = W.Lognormal(1e-2, 0.6, 6.0)
    zh = lattice.forward(field.gaussian_zeta(N, L, 11, spec), L)
    n2 = lattice.n2_half(N)
    w = lattice.half_weights(N)
    k = math.sqrt(1.0) * np.sqrt(n2)
    V = L ** 3
    chi2, dof = 0.0, 0
    for b in range(2, 20):
        m = (k >= b - 0.5) & (k < b + 0.5)
        Pm = field.power_spectrum(k[m], spec.A, spec.sigma, spec.k_star)
        # |zeta_hat|^2 / V is exponentially distributed with mean P(k) per mode
        ratio = np.abs(zh[m]) ** 2 / V / Pm
        nmodes = w[m].sum() / 2.0   # independent complex modes
        est = np.sum(w[m] * ratio) / w[m].sum()
        chi2 += (est - 1.0) ** 2 * nmodes
        dof += 1
    assert chi2 / dof < 3.0


def test_zeta_variance_is_lattice_integral():
    N, L = 64, 2 * math.pi
    spec = W.Lognormal(1e-2, 0.5, 6.0)
    zg = field.gaussian_zeta(N, L, 3, spec)
    n2 = lattice.n2_half(N)
    P = np.where(n2 > 0, field.power_spectrum(np.sqrt(n2.astype(float)), spec.A, spec.sigma,
                                              spec.k_star), 0.0)
    expect = np.sum(lattice.half_weights(N) * P) / L ** 3
    assert abs(expect - spec.A) < 0.05 * spec.A          # lattice sum ~ int Delta^2 dln k
    assert zg.var() == pytest.approx(expect, rel=0.1)    # one realisation, cosmic variance
    assert abs(zg.mean()) < 1e-15                        # k = 0 mode removed


def test_phi_hat_definition_and_hermitian():
    N, L = 16, 2 * math.pi
    spec = W.Lognormal(1e-2, 0.5, 4.0)
    zg = field.gaussian_zeta(N, L, 0, spec)
    ph = field.phi_hat_from_zeta(zg, L)
    full = np.fft.fftn(zg) * (L / N) ** 3 * 2.0 / 3.0
    np.testing.assert_allclose(ph, full[: N // 2 + 1], atol=1e-15)


def test_maps():
    N, L = 32, 2 * math.pi
    spec = W.Lognormal(1e-2, 0.5, 6.0)
    zg = field.gaussian_zeta(N, L, 1, spec)
    loc = field.apply_map(zg, W.NGMap("local", F_NL=3.0, G_NL=2.0))
    m2 = np.mean(zg * zg)
    np.testing.assert_allclose(loc, zg + 3.0 * (zg * zg - m2) + 2.0 * zg ** 3, rtol=1e-15)
    assert abs(np.mean(loc - zg - 2.0 * zg ** 3)) < 1e-16
    ex = field.apply_map(zg, W.NGMap("exptail", beta=3.0, clip=1e-6))
    ok = 1.0 - 3.0 * zg > 1e-6
    assert ok.sum() > 0.9 * ok.size
    np.testing.assert_allclose(ex[ok], -np.log1p(-3.0 * zg[ok]) / 3.0, rtol=0, atol=1e-15)
    np.testing.assert_allclose(ex[~ok], -math.log(1e-6) / 3.0, rtol=1e-15)
    big = np.array([[[0.5, 0.1]]])
    out = field.apply_map(big, W.NGMap("exptail", beta=3.0, clip=1e-6))
    assert out[0, 0, 0] == pytest.approx(-math.log(1e-6) / 3.0)
    assert out[0, 0, 1] == pytest.approx(-math.log(0.7) / 3.0)


# ------------------------------------------------------------- non-local map
def _grid(N, L):
    x = np.arange(N) * (L / N)
    return np.meshgrid(x, x, x, indexing="ij")


def test_nonlocal_map_reduces_to_gaussian():
    zg = field.gaussian_zeta(16, 2 * math.pi, 3, W.Lognormal(1e-2, 0.5, 3.0))
    m = W.NGMap("nonlocal", alpha_NL=0.0, beta_NL=0.0, k_NL=3.0)
    np.testing.assert_array_equal(field.apply_map(zg, m, 2 * math.pi), zg)


def test_nonlocal_map_plane_wave_closed_form():
    """Eq. nonlocal for zeta_g = A cos(q.x): lap(zeta_g^2) = -2|q|^2 A^2 cos(2 q.x)
    and zeta_g lap(zeta_g) = -|q|^2 A^2 cos^2(q.x), in a box with k_F = 0.5."""
    N, L, A = 16, 4 * math.pi, 0.3
    n = np.array([2, -1, 3])                       # 2n stays inside [-N/2, N/2)
    q = n * (2 * math.pi / L)
    X, Y, Z = _grid(N, L)
    ph = q[0] * X + q[1] * Y + q[2] * Z
    zg = A * np.cos(ph)
    a, b, kn = 0.7, -1.3, 3.0
    got = field.apply_map(zg, W.NGMap("nonlocal", alpha_NL=a, beta_NL=b, k_NL=kn), L)
    qq = float(q @ q)
    ref = zg + a / kn ** 2 * (-2 * qq * A * A * np.cos(2 * ph)) + b / kn ** 2 * (-qq * A * A * np.cos(ph) ** 2)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


def _fd4_laplacian(F, h):
    """Fourth-order central differences, periodic."""
    out = np.zeros_like(F)
    for ax in range(3):
        out += (-np.roll(F, 2, ax) + 16 * np.roll(F, 1, ax) - 30 * F + 16 * np.roll(F, -1, ax)
                - np.roll(F, -2, ax)) / (12 * h * h)
    return out


def _fd4_grad2(F, h):
    g2 = np.zeros_like(F)
    for ax in range(3):
        d = (-np.roll(F, -2, ax) + 8 * np.roll(F, -1, ax) - 8 * np.roll(F, 1, ax) + np.roll(F, 2, ax)) / (12 * h)
        g2 += d * d
    return g2


def test_nonlocal_laplacian_against_finite_differences():
    """A smooth field (modes |n_i| <= 2 only) on 48^3: the spectral Laplacian
    of zeta_g^2 and of zeta_g agrees with fourth-order finite differences, and
    the mean of zeta_g lap(zeta_g) equals -mean |grad zeta_g|^2 (integration
    by parts, gradient by finite differences)."""
    N, L = 48, 2 * math.pi
    h = L / N
    rs = np.random.Generator(np.random.PCG64(11))
    X, Y, Z = _grid(N, L)
    zg = np.zeros((N, N, N))
    for _ in range(6):
        n = rs.integers(-2, 3, size=3)
        zg += rs.normal() * np.cos(n[0] * X + n[1] * Y + n[2] * Z + rs.uniform(0, 2 * math.pi))
    for F in (zg, zg * zg):
        lap = field.laplacian(F, L)
        fd = _fd4_laplacian(F, h)
        assert np.max(np.abs(lap - fd)) <= 2e-3 * np.max(np.abs(lap))
    lhs = float(np.mean(zg * field.laplacian(zg, L)))
    rhs = -float(np.mean(_fd4_grad2(zg, h)))
    assert abs(lhs - rhs) <= 2e-3 * abs(rhs)
    # the map itself is the stated combination of the two
    m = W.NGMap("nonlocal", alpha_NL=0.4, beta_NL=0.9, k_NL=2.0)
    got = field.apply_map(zg, m, L)
    ref = zg + 0.4 / 4.0 * _fd4_laplacian(zg * zg, h) + 0.9 / 4.0 * zg * _fd4_laplacian(zg, h)
    assert np.max(np.abs(got - ref)) <= 2e-3 * np.max(np.abs(got - zg))
