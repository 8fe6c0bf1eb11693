"""Physics pins of the whole oracle chain.

P4  Gaussian log-normal (A = 1e-2, sigma = 0.5, k* = 6) on 64^3 with L = 2 pi:
    the four-seed mean of the lattice Omega agrees with the semi-analytic
    Eq. semi_anal within 10% at k/k* = 0.5, 1, 1.15, 1.5, 2 (the accuracy the
    paper reports at N = 64 with 50 kept modes, Sec. VI A and VII).  A missing
    factor 2, 4 or 16/81 anywhere in the chain would fail this by far.
    The two sides are independent computations (lattice FFT chain versus a
    2D quadrature of the printed T(q, s)), so their agreement pins both; the
    quadrature is further checked for its exact A^2 scaling, its dependence
    on k/k* only, and the zero of T(q, s) on the kinematic boundary s = 1.
P4' the paper's other peak widths (Sec. VI A, Fig. Gaussian), with its
    per-target box (Sec. VI: L_k = pi N / (3 max(k, k_bar)), eps = 0.1) at
    64^3 and four seeds, against Eq. semi_anal evaluated with a finer split:
    sigma = 0.1 (k* = 10) within 10% at seven points across the peak and the
    resonance spike; sigma = 1 within 10% for k/k* >= 1.15, while at
    k/k* = 0.5 and 1 the measured miss is 26% and 15% (the box k_max =
    3 k_bar puts k* at 3 k_F: those shells hold 26 and 90 modes and about
    14% of the peak's power lies below k_F), pinned at 30%.
P3  the decomposition error: the oracle against the direct mode sum with the
    exact closed-form kernels (no wrap, same target k, same triangle strip)
    on 24^3; report-level check of the 50-term truncation on the total
    (sine + cosine) shell power.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import adaptive, bruteforce, decomposition, field, lattice, semianalytic, spectrum


@pytest.fixture(scope="module")
def tabs():
    return decomposition.tables()


def test_semianalytic_kernel_limits():
    # T(q,s) vanishes at the kinematic boundary s = 1 and is finite below resonance
    assert semianalytic.T_kernel(0.3, 1.0) == 0.0
    assert np.isfinite(semianalytic.T_kernel(0.5, 1.5))
    # scaling: Omega is quadratic in the amplitude A
    o1 = semianalytic.omega_gauss(6.0, 1.0, 0.5, 6.0, epsrel=1e-7)
    o2 = semianalytic.omega_gauss(6.0, 2.0, 0.5, 6.0, epsrel=1e-7)
    assert o2 == pytest.approx(4 * o1, rel=1e-6)
    # self-similarity: Omega depends on k/k* only
    o3 = semianalytic.omega_gauss(12.0, 1.0, 0.5, 12.0, epsrel=1e-7)
    assert o3 == pytest.approx(o1, rel=1e-6)


@pytest.mark.slow
def test_lattice_matches_semianalytic_gaussian(tabs):
    N, L = 64, 2 * math.pi
    spec = W.Lognormal(1e-2, 0.5, 6.0)
    xs = np.array([0.5, 1.0, 1.15, 1.5, 2.0])
    targets = xs * spec.k_star
    lo, hi = W.thin_shells(targets, L)
    semi = np.array([semianalytic.omega_gauss(k, spec.A, spec.sigma, spec.k_star) for k in targets])
    runs = []
    for seed in range(4):
        ph = field.phi_hat(N, L, seed, spec, W.NGMap())
        om, nb = spectrum.omega_spectrum(ph, tabs[0], tabs[1], targets, lo, hi, L)
        runs.append(om)
    ratio = np.mean(runs, axis=0) / semi
    assert np.all(np.abs(ratio - 1.0) < 0.10), ratio


def test_semianalytic_split_does_not_change_the_result():
    for sigma, x in ((0.5, 1.15), (0.1, 1.0), (1.0, 0.5)):
        a = semianalytic.omega_gauss(6.0 * x, 1.0, sigma, 6.0, epsrel=1e-9)
        b = semianalytic.omega_gauss(6.0 * x, 1.0, sigma, 6.0, epsrel=1e-9, pieces=30)
        assert b == pytest.approx(a, rel=1e-6), (sigma, x)


@pytest.mark.slow
@pytest.mark.parametrize("sigma,xs,tols", [
    (0.1, (0.5, 0.8, 1.0, 1.1, 1.15, 1.3, 1.5), (0.10,) * 7),
    (1.0, (0.5, 1.0, 1.15, 1.5, 2.0), (0.30, 0.30, 0.10, 0.10, 0.10)),
])
def test_lattice_matches_semianalytic_other_widths(tabs, sigma, xs, tols):
    spec = W.Lognormal(1e-2, sigma, 10.0)
    ks = np.array(xs) * spec.k_star
    got = np.zeros(len(ks))
    for seed in range(4):
        got += np.array([o for o, _, _ in adaptive.omega_adaptive(64, seed, spec, W.NGMap("gauss"), ks,
                                                                   tabs=tabs)]) / 4
    ref = np.array([semianalytic.omega_gauss(k, spec.A, spec.sigma, spec.k_star, pieces=30) for k in ks])
    ratio = got / ref
    print("sigma", sigma, "lattice / semi-analytic", np.round(ratio, 3), flush=True)
    assert np.all(np.abs(ratio - 1.0) <= np.array(tols)), ratio


def test_decomposition_error_against_exact_kernels(tabs):
    N, L = 24, 2 * math.pi
    spec = W.Lognormal(1e-2, 0.5, 5.0)
    ph = field.phi_hat(N, L, 1, spec, W.NGMap())
    k_b = 5.0
    n2 = lattice.n2_half(N)
    sel = np.argwhere((n2 > 0) & (np.sqrt(n2) >= k_b - 0.5) & (np.sqrt(n2) < k_b + 0.5))
    modes = [tuple(int(i) for i in s) for s in sel]
    nx, ny, nz = lattice.mode_grids_half(N)
    vec = np.array([[nx[a, 0, 0], ny[0, b, 0], nz[0, 0, c]] for (a, b, c) in modes], float)
    khat = vec / np.linalg.norm(vec, axis=1)[:, None]
    w = np.array([lattice.half_weights(N)[a, b, c] for (a, b, c) in modes])
    p_got = p_ex = 0.0
    for tab, which in ((tabs[0], "s"), (tabs[1], "c")):
        Q = spectrum.source_qhat(ph, tab, k_b, L)
        got = np.stack([Q[:, a, b, c] for (a, b, c) in modes], axis=1)
        ex = bruteforce.exact_qhat(ph, which, L, modes, k_b)
        p_got += np.sum(w * spectrum.tt_power(spectrum.sym3(got), khat))
        p_ex += np.sum(w * spectrum.tt_power(spectrum.sym3(ex), khat))
    # the 50-term kernel changes the shell power by a modest fraction only
    assert abs(p_got / p_ex - 1.0) < 0.25, p_got / p_ex


# ------------------------------------------------------------- per-target box


def test_kbar_against_normal_quantile():
    """The log-normal Delta^2 is a Gaussian in log k, so k_bar = k* exp(sigma z)
    with z the standard normal quantile of 1 - eps (scipy.stats)."""
    from scipy import stats
    for spec, eps in ((W.Lognormal(1e-2, 0.5, 20.0), 0.1), (W.Lognormal(5e-3, 0.3, 40.0), 0.05),
                      (W.Lognormal(1.0, 1.2, 3.0), 0.2)):
        kb = adaptive.k_bar(spec, eps)
        ref = spec.k_star * math.exp(spec.sigma * stats.norm.ppf(1.0 - eps))
        assert abs(kb - ref) <= 1e-10 * ref
        L = adaptive.box_for_target(64, 0.5 * spec.k_star, spec, eps)
        assert abs(L - math.pi * 64 / (3 * ref)) <= 1e-10 * L      # k below k_bar: k_bar sets the box
        L2 = adaptive.box_for_target(64, 10 * spec.k_star, spec, eps)
        assert abs(L2 - math.pi * 64 / (30 * spec.k_star)) <= 1e-12 * L2


def test_adaptive_protocol_against_semi_analytic():
    """Gaussian log-normal sigma = 0.5 at 64^3 with the per-target box: three
    targets around the peak within 20% of Eq. semi_anal (averaged over 3 seeds)."""
    spec = W.Lognormal(1e-2, 0.5, 10.0)
    ks = np.array([7.0, 11.5, 16.0])
    tabs = decomposition.tables()
    got = np.zeros(len(ks))
    for seed in range(3):
        got += np.array([o for o, _, _ in adaptive.omega_adaptive(64, seed, spec, W.NGMap("gauss"), ks,
                                                                   tabs=tabs)]) / 3
    ref = np.array([semianalytic.omega_gauss(k, spec.A, spec.sigma, spec.k_star) for k in ks])
    rel = np.abs(got - ref) / ref
    assert np.all(rel < 0.2), rel
