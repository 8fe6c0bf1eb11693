"""Pins of the per-target convolution engine, TT projection and shell average.

P1  FFT engine == direct O(N^6) mode sum with the kept separable kernel and
    the periodic wrap (Eq. naive_A/B in discrete form), on 8^3 and 16^3, for
    both kernels, every output mode of several shells: 1e-12.
P2  two-plane-wave worked example: with Phi_hat nonzero only at +-p1, +-p2,
    Q_hat(p1+p2) = -(1/V) [qt(p1) qt(p2)^T + qt(p2) qt(p1)^T] K(u1,u2) Phi(p1) Phi(p2)
    and Q_hat(2 p1) = -(1/V) qt(p1) qt(p1)^T K(u1,u1) Phi(p1)^2, in closed form.
P8  the Lambda form of sum_lambda |e^lambda : X|^2 equals the explicit
    polarisation tensors of Sec. I (u-hat = k x x-hat normalised, v = k x u),
    is invariant under rotating u-hat, and Y - P tr(Y)/2 is transverse-traceless.
P9  half-spectrum weighted shell sums equal full-grid sums; N_b counts.
P10 translation, axis permutation and reflection of zeta leave Omega unchanged.
P11 zeta -> zeta + c leaves Omega unchanged; zeta -> c zeta scales Omega by c^4;
    local map with F = G = 0 is the Gaussian case; the exponential tail agrees
    with its Taylor expansion (F_NL = beta/2, G_NL = beta^2/3) at small amplitude.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import bruteforce, decomposition, field, lattice, spectrum


@pytest.fixture(scope="module")
def tabs():
    return decomposition.tables()


def _phi(N, seed=0, spec=W.Lognormal(1e-2, 0.5, 3.0), ngmap=W.NGMap()):
    return field.phi_hat(N, 2 * math.pi, seed, spec, ngmap)


@pytest.mark.parametrize("N,k_b", [(8, 2.0), (16, 3.0), (16, 5.5)])
def test_fft_engine_equals_bruteforce(tabs, N, k_b):
    L = 2 * math.pi
    ph = _phi(N, seed=N, spec=W.Lognormal(1e-2, 0.5, k_b))
    n = lattice.signed_full(N)
    for tab in tabs:
        Q = spectrum.source_qhat(ph, tab, k_b, L)
        # every half-layout mode with |n| in a band around the target
        n2 = lattice.n2_half(N)
        sel = np.argwhere((n2 > 0) & (np.sqrt(n2) >= k_b - 1.5) & (np.sqrt(n2) < k_b + 1.5))
        modes = [tuple(int(i) for i in s) for s in sel[:: max(1, len(sel) // 120)]]
        ref = bruteforce.truncated_qhat(ph, tab, k_b, L, modes)
        got = np.stack([Q[:, a, b, c] for (a, b, c) in modes], axis=1)
        scale = np.max(np.abs(ref))
        assert np.max(np.abs(got - ref)) <= 1e-12 * scale


def test_two_plane_waves_closed_form(tabs):
    N, L = 16, 2 * math.pi
    V = L ** 3
    k_b = 3.0
    p1, p2 = (1, 2, 0), (2, -1, 1)
    ph = np.zeros(lattice.half_shape(N), dtype=np.complex128)
    a1, a2 = 0.7 - 0.2j, -0.3 + 0.9j
    ph[p1[0], p1[1] % N, p1[2] % N] = a1
    ph[p2[0], p2[1] % N, p2[2] % N] = a2
    qt = lambda p: np.array(p, dtype=float)  # k_F = 1, no Nyquist component here
    u1 = math.sqrt(sum(x * x for x in p1)) / k_b
    u2 = math.sqrt(sum(x * x for x in p2)) / k_b
    for tab in tabs:
        i1, i2 = tab.interval_index(np.array([u1, u2]))
        K12 = float(np.sum(tab.sigma * tab.phi[i1] * tab.phi[i2]))
        K11 = float(np.sum(tab.sigma * tab.phi[i1] * tab.phi[i1]))
        Q = spectrum.source_qhat(ph, tab, k_b, L)
        s = tuple(a + b for a, b in zip(p1, p2))
        got = spectrum.sym3(Q[:, s[0], s[1] % N, s[2] % N][:, None])[0]
        ref = -(np.outer(qt(p1), qt(p2)) + np.outer(qt(p2), qt(p1))) * K12 * a1 * a2 / V
        np.testing.assert_allclose(got, ref, rtol=0, atol=1e-13 * np.max(np.abs(ref)))
        d = tuple(2 * a for a in p1)
        got2 = spectrum.sym3(Q[:, d[0], d[1] % N, d[2] % N][:, None])[0]
        ref2 = -np.outer(qt(p1), qt(p1)) * K11 * a1 * a1 / V
        np.testing.assert_allclose(got2, ref2, rtol=0, atol=1e-13 * np.max(np.abs(ref2)))
        # a mode no pair reaches is empty
        assert np.max(np.abs(Q[:, 5, 5, 5])) < 1e-15 * np.max(np.abs(ref))


def _explicit_pol_power(X, khat):
    out = []
    for Xm, k in zip(X, khat):
        ex = np.array([1.0, 0.0, 0.0])
        c = np.cross(k, ex)
        if np.linalg.norm(c) < 1e-12:
            c = np.cross(k, np.array([0.0, 1.0, 0.0]))
        u = c / np.linalg.norm(c)
        v = np.cross(k, u)
        ep = (np.outer(u, u) - np.outer(v, v)) / math.sqrt(2)
        ec = (np.outer(u, v) + np.outer(v, u)) / math.sqrt(2)
        out.append(abs(np.sum(ep * Xm)) ** 2 + abs(np.sum(ec * Xm)) ** 2)
    return np.array(out)


def test_tt_projection_matches_polarisation_tensors():
    r = np.random.default_rng(5)
    M = 200
    A = r.standard_normal((M, 3, 3)) + 1j * r.standard_normal((M, 3, 3))
    X = A + np.transpose(A, (0, 2, 1))
    k = r.standard_normal((M, 3))
    k[0] = [1.0, 0.0, 0.0]           # k-hat along x: the special case of the basis
    k[1] = [0.0, 0.0, -2.0]
    khat = k / np.linalg.norm(k, axis=1)[:, None]
    np.testing.assert_allclose(spectrum.tt_power(X, khat), _explicit_pol_power(X, khat), rtol=1e-12)
    # rotating u-hat by psi mixes + and x but leaves the sum unchanged
    for j in range(5):
        kk = khat[j]
        u = np.cross(kk, [0.3, 0.5, 0.8]); u /= np.linalg.norm(u)
        v = np.cross(kk, u)
        tot = []
        for psi in (0.0, 0.4, 1.3):
            uu = math.cos(psi) * u + math.sin(psi) * v
            vv = np.cross(kk, uu)
            ep = (np.outer(uu, uu) - np.outer(vv, vv)) / math.sqrt(2)
            ec = (np.outer(uu, vv) + np.outer(vv, uu)) / math.sqrt(2)
            tot.append(abs(np.sum(ep * X[j])) ** 2 + abs(np.sum(ec * X[j])) ** 2)
        np.testing.assert_allclose(tot, tot[0], rtol=1e-12)
    # transverse-traceless part
    P = np.eye(3)[None] - khat[:, :, None] * khat[:, None, :]
    Y = P @ X @ P
    Pi = Y - 0.5 * P * np.trace(Y, axis1=1, axis2=2)[:, None, None]
    assert np.max(np.abs(np.einsum("mi,mij->mj", khat, Pi))) < 1e-12
    assert np.max(np.abs(np.trace(Pi, axis1=1, axis2=2))) < 1e-12


def test_half_layout_shell_sums_equal_full_grid(tabs):
    N, L = 16, 2 * math.pi
    ph = _phi(N, seed=4, spec=W.Lognormal(1e-2, 0.5, 4.0))
    k_b, lo, hi = 4.0, 3.5, 4.5
    Qs = spectrum.source_qhat(ph, tabs[0], k_b, L)
    Qc = spectrum.source_qhat(ph, tabs[1], k_b, L)
    S, Nb = spectrum.shell_sum(Qs, Qc, k_b, lo, hi, L)
    # full grid
    n = lattice.signed_full(N)
    full_s = np.stack([bruteforce.full_from_half(Qs[c]) for c in range(6)])
    full_c = np.stack([bruteforce.full_from_half(Qc[c]) for c in range(6)])
    nx, ny, nz = np.meshgrid(n, n, n, indexing="ij")
    kk = np.sqrt(nx ** 2 + ny ** 2 + nz ** 2)
    m = (kk >= lo) & (kk < hi)
    vec = np.stack([nx[m], ny[m], nz[m]], axis=1).astype(float)
    khat = vec / np.linalg.norm(vec, axis=1)[:, None]
    pref = 4.0 / k_b ** 2
    s = spectrum.tt_power(spectrum.sym3(-pref * full_s[:, m]), khat) + \
        spectrum.tt_power(spectrum.sym3(pref * full_c[:, m]), khat)
    assert Nb == int(m.sum())
    assert S == pytest.approx(float(s.sum()), rel=1e-12)


def test_mode_counts_partition():
    N, L = 32, 2 * math.pi
    e, t = W.linear_bins(N, L, 16)
    lo, hi = W.shells_from_edges(e)
    nb = spectrum.mode_counts(N, L, lo, hi)
    n = lattice.signed_full(N)
    nx, ny, nz = np.meshgrid(n, n, n, indexing="ij")
    kk = np.sqrt(nx ** 2 + ny ** 2 + nz ** 2)
    assert nb.sum() == int(((kk >= e[0]) & (kk < e[-1])).sum())
    assert nb[0] == 18   # |n| in [0.5, 1.5): the 6 axis and 12 face-diagonal neighbours


def _omega(ph, tabs, targets, lo, hi, L=2 * math.pi):
    om, nb = spectrum.omega_spectrum(ph, tabs[0], tabs[1], targets, lo, hi, L)
    return om


def test_symmetries_of_the_pipeline(tabs):
    N, L = 16, 2 * math.pi
    spec = W.Lognormal(1e-2, 0.5, 3.0)
    zg = field.gaussian_zeta(N, L, 2, spec)
    targets = np.array([2.0, 3.0, 4.5])
    lo, hi = targets - 0.5, targets + 0.5
    base = _omega(field.phi_hat_from_zeta(zg, L), tabs, targets, lo, hi)
    assert np.all(base > 0)
    variants = [np.roll(zg, (3, -5, 7), axis=(0, 1, 2)),
                np.transpose(zg, (1, 2, 0)), np.transpose(zg, (2, 1, 0)),
                zg[::-1, :, :], zg[:, ::-1, ::-1]]
    for v in variants:
        om = _omega(field.phi_hat_from_zeta(np.ascontiguousarray(v), L), tabs, targets, lo, hi)
        np.testing.assert_allclose(om, base, rtol=1e-11)


def test_map_properties(tabs):
    N, L = 16, 2 * math.pi
    spec = W.Lognormal(1e-2, 0.5, 3.0)
    zg = field.gaussian_zeta(N, L, 9, spec)
    targets = np.array([2.0, 3.5])
    lo, hi = targets - 0.5, targets + 0.5
    om = lambda z: _omega(field.phi_hat_from_zeta(z, L), tabs, targets, lo, hi)
    base = om(zg)
    np.testing.assert_allclose(om(zg + 0.37), base, rtol=1e-11)
    np.testing.assert_allclose(om(2.5 * zg), base * 2.5 ** 4, rtol=1e-11)
    loc0 = field.apply_map(zg, W.NGMap("local", F_NL=0.0, G_NL=0.0))
    np.testing.assert_allclose(om(loc0), base, rtol=1e-13)
    # exponential tail -> local with its Taylor coefficients at small amplitude
    small = zg * 1e-2
    beta = 3.0
    g = om(small)
    ex = om(field.apply_map(small, W.NGMap("exptail", beta=beta, clip=1e-6)))
    lc = om(field.apply_map(small, W.NGMap("local", F_NL=beta / 2, G_NL=beta ** 2 / 3)))
    assert np.all(np.abs(ex - g) > 1e-4 * g)            # the non-Gaussian part is visible
    np.testing.assert_allclose(ex - g, lc - g, rtol=2e-3)


# --------------------------------------------------------------- jackknife
from oracle import jackknife  # noqa: E402


def _random_hermitian_qhat(N, seed):
    """Six half spectra that are DFTs of real fields (so Hermitian)."""
    rs = np.random.Generator(np.random.PCG64(seed))
    return np.stack([lattice.forward(rs.normal(size=(N, N, N)), 2 * np.pi) for _ in range(6)])


def test_jackknife_sums_reproduce_shell_sum():
    """Parseval: the sub-volume sums of the real-space TT fields add up to the
    shell estimator's S_b (computed mode by mode), and the replica mean is Omega."""
    N, L, M = 16, 2 * np.pi, 4
    Qs, Qc = _random_hermitian_qhat(N, 1), _random_hermitian_qhat(N, 2)
    for k_b, lo, hi in ((3.0, 2.5, 3.5), (5.2, 4.6, 5.9)):
        h = jackknife.shell_tt_fields(Qs, Qc, k_b, lo, hi, L)
        S_i = jackknife.subvolume_sums(h, L, M)
        S_b, N_b = spectrum.shell_sum(Qs, Qc, k_b, lo, hi, L)
        assert abs(S_i.sum() - S_b) <= 1e-12 * S_b
        om, sigma, rep = jackknife.jackknife_from_sums(S_i, N_b, k_b, L)
        assert abs(rep.mean() - om) <= 1e-12 * om and sigma > 0
        assert abs(om - spectrum.omega_from_sum(S_b, N_b, k_b, L)) <= 1e-12 * om


def test_jackknife_fields_by_direct_sum():
    """The real-space fields against an explicit sum over the shell's full-grid
    modes with the projector built from the explicit e^+, e^x tensors' sum
    (sum_lambda e^lambda_ij e^lambda_lm = Lambda_ij,lm) on 8^3."""
    N, L = 8, 2 * np.pi
    Qs, Qc = _random_hermitian_qhat(N, 3), _random_hermitian_qhat(N, 4)
    k_b, lo, hi = 2.4, 2.0, 3.0
    h = jackknife.shell_tt_fields(Qs, Qc, k_b, lo, hi, L)
    x = np.arange(N) * (L / N)
    X_, Y_, Z_ = np.meshgrid(x, x, x, indexing="ij")
    nx, ny, nz = lattice.mode_grids_full(N)
    ref = np.zeros((2, 3, 3, N, N, N), dtype=np.complex128)
    for m, (Q, sign) in enumerate(((Qs, -1.0), (Qc, 1.0))):
        for a in range(N):
            for b in range(N):
                for c in range(N):
                    n = np.array([nx[a, 0, 0], ny[0, b, 0], nz[0, 0, c]], dtype=np.float64)
                    kk = np.linalg.norm(n)
                    if kk == 0 or not (lo <= kk < hi):
                        continue
                    # X(n) from the half layout (conjugate for kx < 0)
                    if n[0] >= 0 and a <= N // 2:
                        Xc = Q[:, a, b, c]
                    else:
                        Xc = np.conj(Q[:, (-a) % N, (-b) % N, (-c) % N])
                    T = np.zeros((3, 3), dtype=np.complex128)
                    for cc, (i, j) in enumerate(spectrum.PAIRS):
                        T[i, j] = T[j, i] = sign * 4.0 / k_b ** 2 * Xc[cc]
                    kh = n / kk
                    Pm = np.eye(3) - np.outer(kh, kh)
                    Lam = 0.5 * (np.einsum("il,jm->ijlm", Pm, Pm) + np.einsum("im,jl->ijlm", Pm, Pm)
                                 - np.einsum("ij,lm->ijlm", Pm, Pm))
                    Yt = np.einsum("ijlm,lm->ij", Lam, T)
                    ph = np.exp(1j * (n[0] * X_ + n[1] * Y_ + n[2] * Z_))
                    ref[m] += Yt[:, :, None, None, None] * ph[None, None] / L ** 3
    assert np.max(np.abs(ref.imag)) <= 1e-12 * np.max(np.abs(ref.real))
    assert np.max(np.abs(h - ref.real)) <= 1e-12 * np.max(np.abs(h))


def test_jackknife_single_commensurate_mode_has_zero_error():
    """One mode pair +-n whose wavelength divides the sub-volume edge: every
    sub-volume holds the same energy, so every replica equals Omega and the
    jackknife error vanishes; a second, incommensurate mode breaks that."""
    N, L, M = 16, 2 * np.pi, 2
    Q = np.zeros((6, N // 2 + 1, N, N), dtype=np.complex128)
    Q[:, 0, 2, 0] = [1.0, 0.5, -0.3, 0.2j, 0.1, -0.4j]          # n = (0, 2, 0): wavelength N/2
    Q[:, 0, N - 2, 0] = np.conj(Q[:, 0, 2, 0])                    # its mirror in the kx = 0 plane
    Z = np.zeros_like(Q)
    h = jackknife.shell_tt_fields(Q, Z, 2.0, 1.5, 2.5, L)
    om, sigma, rep = jackknife.jackknife_from_sums(jackknife.subvolume_sums(h, L, M), 2, 2.0, L)
    assert om > 0 and sigma <= 1e-12 * om
    # two modes n = (1, 0, 0) and (0, 1, 0) of one shell: their interference
    # cos(2 pi (x - y) / N) puts different energy into different sub-volumes
    Q2 = np.zeros_like(Q)
    Q2[:, 1, 0, 0] = [0.3, 0.2, 0.5, 0.0, 0.05, 0.1]
    Q2[:, 0, 1, 0] = [0.2, 0.1, 0.4, 0.0, 0.1, 0.0]
    Q2[:, 0, N - 1, 0] = np.conj(Q2[:, 0, 1, 0])
    h = jackknife.shell_tt_fields(Q2, Z, 1.0, 0.5, 1.5, L)
    S_i = jackknife.subvolume_sums(h, L, M)
    om, sigma, rep = jackknife.jackknife_from_sums(S_i, 4, 1.0, L)
    assert sigma > 1e-3 * om and np.ptp(S_i) > 1e-3 * S_i.mean()
    with pytest.raises(ValueError):
        jackknife.subvolume_sums(h, L, 3)
    with pytest.raises(ValueError):
        jackknife.shell_tt_fields(Q, Z, 8.0, 7.5, 8.5, L)


def test_decompose_other_kernel_reconstructs_it():
    """The decomposition of Sec. V applied to another kernel (a callable on
    the same strip) keeps its meaning: with every term kept it reproduces
    the kernel matrix on the interval centres exactly, and the plain call is
    the kernel=None path."""
    def toy(u, v):
        return np.cos(1.3 * u) * np.cos(0.7 * v) + np.cos(0.7 * u) * np.cos(1.3 * v)
    t = decomposition.decompose("s", n_modes=40, n_alpha=40, u_max=6.0, kernel=toy)
    c = 0.5 * (t.edges[:-1] + t.edges[1:])
    U, V = np.meshgrid(c, c, indexing="ij")
    strip = (np.abs(U - V) <= 1.0) & (U + V >= 1.0)
    K = np.where(strip, toy(U, V), 0.0)
    assert np.max(np.abs(t.reconstruct() - K)) <= 1e-12 * np.max(np.abs(K))
    a = decomposition.decompose("c", n_modes=30, n_alpha=10)
    b = decomposition.decompose("c", n_modes=30, n_alpha=10, kernel=None)
    np.testing.assert_array_equal(a.phi, b.phi)
