"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Bars (each written in the test):
* white noise: bit-exact (FP64 deviates; FP32 = the FP64 deviate rounded);
* FP64 path: Phi_hat and Q_hat within 1e-12 / 1e-11 of the largest
  magnitude, Omega within 1e-10 relative per non-empty bin, N_b exact;
* FP32 path (complex64 fields/FFTs, FP64 maps and shell sums): Omega within
  1e-4 relative per non-empty bin of the FP64 oracle, N_b exact.
Sizes span several tiles and ragged tails (N = 8 ... 512, radix 3 at 384).
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import decomposition, field, lattice, rng, spectrum

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2605_27231_amd")


@pytest.fixture(scope="module")
def tabs():
    return decomposition.tables()


def _tabs_n(n_alpha):
    return (decomposition.decompose("s", n_alpha=n_alpha), decomposition.decompose("c", n_alpha=n_alpha))


def _np(t):
    return t.detach().cpu().numpy()


def _say(*a):
    print(*a, flush=True)


# ---------------------------------------------------------------- white noise
@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("seed", [0, 7, 2 ** 63 + 5])
def test_white_noise_bit_exact(prec, seed):
    N = 32
    _say(f"noise N={N} prec={prec} seed={seed}")
    with P.Plan(N, prec=prec) as pl:
        got = _np(pl.white_noise(seed))
    ref = rng.white_noise(N, seed)
    if prec == "f32":
        ref = ref.astype(np.float32)
    assert got.dtype == ref.dtype
    np.testing.assert_array_equal(got.view(np.uint64 if prec == "f64" else np.uint32),
                                  ref.view(np.uint64 if prec == "f64" else np.uint32))


# ------------------------------------------------------------ Phi_hat and FFTs
@pytest.mark.parametrize("N", [8, 16, 32, 64, 128, 384])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_phi_hat_from_zeta(N, prec):
    _say(f"set_zeta N={N} prec={prec}")
    L = 2 * math.pi
    z = np.random.default_rng(N).standard_normal((N, N, N))
    if prec == "f32":
        z = z.astype(np.float32).astype(np.float64)
    ref = field.phi_hat_from_zeta(z, L)
    with P.Plan(N, prec=prec) as pl:
        pl.set_zeta(0, torch.from_numpy(z))
        got = _np(pl.get_phi_hat(0)).astype(np.complex128)
    tol = 1e-12 if prec == "f64" else 3e-6
    assert np.max(np.abs(got - ref)) <= tol * np.max(np.abs(ref))


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("ngmap,L", [
    (W.NGMap("gauss"), 2 * math.pi), (W.NGMap("local", F_NL=3.0, G_NL=1.0), 2 * math.pi),
    (W.NGMap("exptail", beta=3.0, clip=1e-6), 2 * math.pi),
    (W.NGMap("nonlocal", alpha_NL=2.0, beta_NL=-3.0, k_NL=6.0), 2 * math.pi),
    (W.NGMap("nonlocal", alpha_NL=-1.5, beta_NL=2.5, k_NL=4.0), 3 * math.pi)],
    ids=["gauss", "local", "exptail", "nonlocal", "nonlocal-L3pi"])
def test_generate_field(prec, ngmap, L):
    N = 64
    spec = W.Lognormal(1e-2, 0.5, 6.0)
    _say(f"generate N={N} prec={prec} map={ngmap.kind}")
    ref = field.phi_hat(N, L, 3, spec, ngmap)
    with P.Plan(N, L=L, prec=prec) as pl:
        pl.generate_field(0, 3, spec, ngmap)
        got = _np(pl.get_phi_hat(0)).astype(np.complex128)
    tol = 1e-11 if prec == "f64" else 2e-5
    assert np.max(np.abs(got - ref)) <= tol * np.max(np.abs(ref))


# ------------------------------------------------------- source convolutions
@pytest.mark.parametrize("N,k_b,prec,n_alpha", [
    (16, 3.0, "f64", 50), (32, 5.5, "f64", 50), (64, 9.0, "f64", 50), (32, 5.5, "f32", 50),
    (128, 20.0, "f32", 6), (256, 30.0, "f32", 6), (384, 50.0, "f32", 2), (384, 50.0, "f64", 2),
    (512, 60.0, "f32", 2), (256, 30.0, "f64", 2)])
def test_source_convolutions(tabs, N, k_b, prec, n_alpha):
    _say(f"qhat N={N} k={k_b} prec={prec} n_alpha={n_alpha}")
    L = 2 * math.pi
    ph = field.phi_hat(N, L, 1, W.Lognormal(1e-2, 0.5, k_b), W.NGMap("local", F_NL=2.0))
    if prec == "f32":
        ph = ph.astype(np.complex64).astype(np.complex128)
    ts = tabs if n_alpha == 50 else _tabs_n(n_alpha)
    with P.Plan(N, prec=prec, n_alpha=n_alpha) as pl:
        pl.set_phi_hat(0, torch.from_numpy(ph))
        got = _np(pl.source_convolutions(0, k_b)).astype(np.complex128)
    tol = 1e-11 if prec == "f64" else 2e-5
    for m in range(2):
        ref = spectrum.source_qhat(ph, ts[m], k_b, L)
        err = np.max(np.abs(got[m] - ref)) / np.max(np.abs(ref))
        assert err <= tol, (m, err)


# ------------------------------------------------------------------ spectra
def _oracle_spectrum(job, tabs, seed, which=None):
    ph = field.phi_hat(job.N, job.L, seed, job.spectrum, job.ngmap)
    return spectrum.omega_spectrum(ph, tabs[0], tabs[1], job.targets, job.k_lo, job.k_hi, job.L, which)


def _check_bins(got, nb, ref, nref, tol):
    np.testing.assert_array_equal(nb, nref)
    ok = nref > 0
    assert np.all(got[~ok] == 0.0)
    rel = np.abs(got[ok] - ref[ok]) / np.abs(ref[ok])
    assert np.max(rel) <= tol, (np.max(rel), np.argmax(rel))
    return rel


def test_spectrum_plain_fp64_32cube(tabs):
    """Gaussian 32^3, A=1e-2, sigma=0.5, k*=6, seed 0, 16 linear bins; FP64: 1e-10 per bin."""
    job = W.config_plain_fp64(32)
    _say("spectrum 32^3 fp64 16 linear bins")
    ref, nref = _oracle_spectrum(job, tabs, 0)
    with P.Plan(32, prec="f64") as pl:
        pl.generate_field(0, 0, job.spectrum, job.ngmap)
        got, nb = pl.spectrum(0, job.targets, job.k_lo, job.k_hi)
    rel = _check_bins(got, nb, ref, nref, 1e-10)
    _say("max rel err per bin", rel.max())


@pytest.mark.parametrize("ngmap", [W.NGMap("local", F_NL=3.0), W.NGMap("exptail", beta=3.0),
                                   W.NGMap("nonlocal", alpha_NL=2.0, beta_NL=-3.0, k_NL=8.0)],
                         ids=["local", "exptail", "nonlocal"])
def test_spectrum_fp32_vs_fp64_oracle(tabs, ngmap):
    """FP32 fields/FFTs with FP64 shell sums against the FP64 oracle: 1e-4 per bin."""
    N, L = 64, 2 * math.pi
    e, t = W.log_bins(N, L, 24)
    lo, hi = W.shells_from_edges(e)
    job = W.Job(N=N, L=L, spectrum=W.Lognormal(1e-2, 0.5, 8.0), ngmap=ngmap, k_lo=lo, k_hi=hi,
                targets=t)
    _say(f"spectrum 64^3 fp32 {ngmap.kind} 24 log bins")
    ref, nref = _oracle_spectrum(job, tabs, 5)
    with P.Plan(N, prec="f32") as pl:
        pl.generate_field(0, 5, job.spectrum, job.ngmap)
        got, nb = pl.spectrum(0, job.targets, job.k_lo, job.k_hi)
    rel = _check_bins(got, nb, ref, nref, 1e-4)
    _say("max rel err per bin", rel.max(), "empty bins", int((nref == 0).sum()))


def test_edge_cases(tabs):
    """8^3 and 16^3 lattices, a shell holding only Nyquist-plane modes, empty
    shells, overlapping shells, no targets, thin shells k +- pi/L."""
    L = 2 * math.pi
    for N in (8, 16):
        ph = field.phi_hat(N, L, 2, W.Lognormal(1e-2, 0.5, 2.5), W.NGMap())
        targets = np.array([2.0, 3.0, 2.5, float(N) / 2, 100.0, 1.0])
        lo = np.array([1.5, 2.5, 1.5, N / 2 * math.sqrt(3) - 1e-9, 99.0, 0.0])
        hi = np.array([2.5, 3.5, 3.5, N / 2 * math.sqrt(3) + 1e-9, 101.0, 0.9])
        _say(f"edge cases N={N}")
        ref, nref = spectrum.omega_spectrum(ph, tabs[0], tabs[1], targets, lo, hi, L)
        with P.Plan(N, prec="f64") as pl:
            pl.set_phi_hat(0, torch.from_numpy(ph))
            got, nb = pl.spectrum(0, targets, lo, hi)
            empty, nbe = pl.spectrum(0, np.zeros(0), np.zeros(0), np.zeros(0))
        assert nref[3] == 1 and nref[4] == 0 and nref[5] == 0   # the Nyquist corner; empty shells
        _check_bins(got, nb, ref, nref, 1e-10)
        assert empty.shape == (0,) and nbe.shape == (0,)


def test_errors_and_state():
    with P.Plan(16, prec="f32", n_slots=2) as pl:
        with pytest.raises(P.SigwError) as e:
            pl.spectrum(1, [2.0], [1.5], [2.5])
        assert e.value.status == -5        # no field in slot 1 yet
        with pytest.raises(P.SigwError) as e:
            pl.spectrum(2, [2.0], [1.5], [2.5])
        assert e.value.status == -1        # slot out of range
        pl.generate_field(1, 0, W.Lognormal(1e-2, 0.5, 3.0), W.NGMap())
        with pytest.raises(P.SigwError) as e:
            pl.spectrum(1, [2.0], [2.5], [1.5])
        assert e.value.status == -1        # k_lo >= k_hi
        with pytest.raises(P.SigwError) as e:
            pl.generate_field(0, 0, W.Lognormal(1e-2, -0.5, 3.0), W.NGMap())
        assert e.value.status == -1
        with pytest.raises(P.SigwError) as e:       # the non-local map needs k_NL > 0
            pl.generate_field(0, 0, W.Lognormal(1e-2, 0.5, 3.0), W.NGMap("nonlocal", alpha_NL=1.0))
        assert e.value.status == -1
        om, nb = pl.spectrum(1, [2.0], [1.5], [2.5])
        assert nb[0] > 0 and om[0] > 0


def test_batch_async_chunking_and_determinism(tabs):
    """A slot's result is the same alone, in a batch, through the asynchronous
    entry points, with fewer terms per workspace pass, and across runs."""
    N, L = 32, 2 * math.pi
    e, t = W.log_bins(N, L, 8)
    lo, hi = W.shells_from_edges(e)
    spec = W.Lognormal(1e-2, 0.6, 5.0)
    with P.Plan(N, prec="f32", n_slots=3) as pl:
        for s in range(3):
            pl.generate_field(s, 10 + s, spec, W.NGMap("local", F_NL=float(s)))
        alone = [pl.spectrum(s, t, lo, hi)[0] for s in range(3)]
        again = [pl.spectrum(s, t, lo, hi)[0] for s in range(3)]
        batch, _ = pl.spectrum_batch([2, 0, 1], t, lo, hi)
        pl.spectrum_enqueue(1, t, lo, hi)
        res = None
        while res is None:
            res = pl.spectrum_poll()
    for s in range(3):
        np.testing.assert_array_equal(alone[s], again[s])
    np.testing.assert_array_equal(batch[0], alone[2])
    np.testing.assert_array_equal(batch[1], alone[0])
    np.testing.assert_array_equal(batch[2], alone[1])
    np.testing.assert_array_equal(res[0], alone[1])
    with P.Plan(N, prec="f32", alpha_chunk=7) as pl:
        pl.generate_field(0, 11, spec, W.NGMap("local", F_NL=1.0))
        chunked = pl.spectrum(0, t, lo, hi)[0]
    ok = alone[1] > 0
    np.testing.assert_allclose(chunked[ok], alone[1][ok], rtol=2e-5)
    # several realisations per launch (groups of 2 over 3 slots: one ragged
    # group) give the same bits as one realisation per launch
    with P.Plan(N, prec="f32", n_slots=3, batch=2) as pl:
        for s in range(3):
            pl.generate_field(s, 10 + s, spec, W.NGMap("local", F_NL=float(s)))
        batched, _ = pl.spectrum_batch([0, 1, 2], t, lo, hi)
        staged, _ = pl.spectrum_batch([1], t, lo, hi)
    for s in range(3):
        np.testing.assert_array_equal(batched[s], alone[s])
    np.testing.assert_array_equal(staged[0], alone[1])
    # staging one term at a time through the (W, Z) scratch changes nothing
    with P.Plan(N, prec="f32", scratch_terms=1) as pl:
        pl.generate_field(0, 11, spec, W.NGMap("local", F_NL=1.0))
        one = pl.spectrum(0, t, lo, hi)[0]
    np.testing.assert_array_equal(one, alone[1])


@pytest.mark.parametrize("N,prec,tol", [(32, "f64", 1e-10), (64, "f32", 1e-4)])
def test_small_supports(tabs, N, prec, tol):
    """Targets whose weighted fields live on a small ball |n| < u_max k_b / k_F
    (u_max = 15): from |n| <= 1 (k_b = 0.07) through supports that end inside
    one FFT radix block or straddle one, to the whole lattice; each with a
    shell of its own and with a fixed shell at |n| = 1..2, so that the rows
    and planes the hot path skips are exercised against the oracle, which
    skips nothing."""
    L = 2 * math.pi
    ph = field.phi_hat(N, L, 4, W.Lognormal(1e-2, 0.7, 3.0), W.NGMap("local", F_NL=2.0))
    if prec == "f32":
        ph = ph.astype(np.complex64).astype(np.complex128)
    kb = np.array([0.07, 0.0667, 0.1, 0.27, 0.55, 0.8, 1.05, 1.6, 2.2, 4.0])
    targets = np.concatenate([kb, kb])
    lo = np.concatenate([np.maximum(kb - 0.5, 0.5), np.full(kb.size, 0.5)])
    hi = np.concatenate([np.maximum(kb + 0.5, 1.5), np.full(kb.size, 2.5)])
    if N > 32:                       # own shells only: keeps the oracle's time down
        targets, lo, hi = targets[:kb.size], lo[:kb.size], hi[:kb.size]
    _say(f"small supports N={N} prec={prec}")
    ref, nref = spectrum.omega_spectrum(ph, tabs[0], tabs[1], targets, lo, hi, L)
    with P.Plan(N, prec=prec) as pl:
        pl.set_phi_hat(0, torch.from_numpy(ph))
        got, nb = pl.spectrum(0, targets, lo, hi)
    assert np.all(nref > 0)
    rel = _check_bins(got, nb, ref, nref, tol)
    _say("max rel err per bin", rel.max())
