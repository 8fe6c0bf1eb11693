"""Jackknife error bars through the C ABI against the FP64 oracle
(oracle/jackknife.py): Omega and N_b as for the plain spectrum, the
jackknife sigma and every replica Omega.  Bars: FP64 path 1e-10 relative on
Omega and the replicas, 1e-8 on sigma; FP32 path 1e-4 on Omega, 1e-3 on
sigma.  Invalid M and shells above the Nyquist frequency are refused."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import decomposition, field, jackknife, spectrum

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2605_27231_amd")
from paper_2605_27231_amd import _lib  # noqa: E402


def _oracle(ph, tabs, targets, lo, hi, L, M):
    out = []
    for k_b, a, b in zip(targets, lo, hi):
        Qs = spectrum.source_qhat(ph, tabs[0], k_b, L)
        Qc = spectrum.source_qhat(ph, tabs[1], k_b, L)
        _, N_b = spectrum.shell_sum(Qs, Qc, k_b, a, b, L)
        S_i = jackknife.subvolume_sums(jackknife.shell_tt_fields(Qs, Qc, k_b, a, b, L), L, M)
        om, sigma, rep = jackknife.jackknife_from_sums(S_i, N_b, k_b, L)
        out.append((om, N_b, sigma, rep))
    return out


@pytest.mark.parametrize("N,prec,M,tol_om,tol_sig", [(32, "f64", 4, 1e-10, 1e-8), (64, "f32", 4, 1e-4, 1e-3),
                                                     (32, "f64", 2, 1e-10, 1e-8)])
def test_jackknife_matches_oracle(N, prec, M, tol_om, tol_sig):
    L = 2 * math.pi
    spec = W.Lognormal(1e-2, 0.5, N / 5)
    ngmap = W.NGMap("local", F_NL=2.0)
    ks = np.array([N / 8, N / 5, N / 3.2])
    lo, hi = ks - math.pi / L, ks + math.pi / L
    print(f"jackknife N={N} {prec} M={M}", flush=True)
    tabs = decomposition.tables()
    ph = field.phi_hat(N, L, 4, spec, ngmap)
    ref = _oracle(ph, tabs, ks, lo, hi, L, M)
    with P.Plan(N, prec=prec) as pl:
        pl.generate_field(0, 4, spec, ngmap)
        om, nb, err, rep = pl.spectrum_jackknife(0, ks, lo, hi, M)
        om_plain, nb_plain = pl.spectrum(0, ks, lo, hi)
    np.testing.assert_array_equal(nb, nb_plain)
    np.testing.assert_array_equal(om, om_plain)
    for b, (o, n, s, r) in enumerate(ref):
        assert nb[b] == n
        assert abs(om[b] - o) <= tol_om * o
        assert abs(err[b] - s) <= tol_sig * s, (b, err[b], s)
        assert np.max(np.abs(rep[b] - r)) <= max(tol_om, 1e-6 if prec == "f32" else 0) * o
        print(f"  k={ks[b]:.2f} Omega={o:.4e} sigma/Omega={s / o:.3f} gpu err rel {abs(err[b] - s) / s:.1e}",
              flush=True)


def test_jackknife_rejects_bad_arguments():
    with P.Plan(32, prec="f32") as pl:
        pl.generate_field(0, 1, W.Lognormal(1e-2, 0.5, 6.0), W.NGMap())
        for M, hi in ((3, 5.5), (1, 5.5), (4, 16.5)):
            with pytest.raises(_lib.SigwError) as e:
                pl.spectrum_jackknife(0, [5.0], [4.5], [hi], M)
            assert e.value.status == _lib.SIGW_E_INVALID
