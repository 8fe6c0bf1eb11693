"""Caller-supplied kernel tables (sigw_plan_set_kernel_table), through the C
ABI: the device path reads only the table, so any separable kernel on any u
grid can stand in for I_s and I_c (Sec. V's decomposition applied to
another kernel, e.g. one from another equation of state).

* the plan's own tables set back unchanged: bit-identical spectra;
* a toy kernel on a wider u grid than the plan was created with (u_max 12
  against 4), decomposed by the oracle: FP64 path within 1e-10 and FP32
  path within 1e-4 per bin of the oracle's spectrum with the same tables
  (the support bound must follow the new grid, or modes would be dropped);
* invalid tables are refused and leave the plan unchanged;
* the tables of a constant equation of state (w = 0.6; Sec. II equations,
  Sec. IV time integrals), built by the oracle and installed: FP64 within
  1e-10 and FP32 within 1e-4 per bin of the oracle's spectrum with the same
  tables; the library's own constant-w tables (Plan.set_equation_of_state)
  within 1e-6 of it (the two builders agree to ~1e-8 in the kept kernel).
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import decomposition, eos, field, spectrum

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2605_27231_amd")
from paper_2605_27231_amd import _lib  # noqa: E402


def _say(*a):
    print(*a, flush=True)


def _toy(u, v):
    # smooth, sign-changing, not separable: stands for a kernel from another cosmology
    return np.cos(1.3 * u) * np.cos(0.7 * v) + np.cos(0.7 * u) * np.cos(1.3 * v) + 0.4 * u * v / (1.0 + u * v)


META = dict(n_modes=120, n_alpha=30, u_min=1e-3, u_p=1.0, sigma_p=0.5, A_p=10.0)


def _job(N):
    L = 2 * math.pi
    e, t = W.log_bins(N, L, 12)
    lo, hi = W.shells_from_edges(e)
    return W.Job(N=N, L=L, spectrum=W.Lognormal(1e-2, 0.6, N / 6.0), ngmap=W.NGMap("local", F_NL=2.0),
                 k_lo=lo, k_hi=hi, targets=t)


def test_own_table_roundtrip():
    job = _job(32)
    _say("own table set back, 32^3 f64")
    with P.Plan(32, prec="f64") as pl:
        pl.generate_field(0, 3, job.spectrum, job.ngmap)
        om0, nb0 = pl.spectrum(0, job.targets, job.k_lo, job.k_hi)
        for m in range(2):
            s, phi, e = P.sigw_kernel_table(pl.desc, m)
            pl.set_kernel_table(m, s, phi, e)
        om1, nb1 = pl.spectrum(0, job.targets, job.k_lo, job.k_hi)
    np.testing.assert_array_equal(nb0, nb1)
    np.testing.assert_array_equal(om0.view(np.uint64), om1.view(np.uint64))


@pytest.mark.parametrize("N,prec,tol", [(32, "f64", 1e-10), (64, "f32", 1e-4)])
def test_custom_kernel_vs_oracle(N, prec, tol):
    job = _job(N)
    tabs = (decomposition.decompose("s", u_max=12.0, kernel=_toy, **META),
            decomposition.decompose("c", u_max=12.0, kernel=lambda u, v: _toy(u, v) * np.exp(-0.1 * (u + v)),
                                    **META))
    ph = field.phi_hat(N, job.L, 4, job.spectrum, job.ngmap)
    _say(f"custom kernel tables N={N} prec={prec}")
    ref, nref = spectrum.omega_spectrum(ph, tabs[0], tabs[1], job.targets, job.k_lo, job.k_hi, job.L)
    with P.Plan(N, prec=prec, u_max=4.0, **META) as pl:
        pl.generate_field(0, 4, job.spectrum, job.ngmap)
        for m in range(2):
            pl.set_kernel_table(m, tabs[m].sigma, tabs[m].phi, tabs[m].edges)
        got, nb = pl.spectrum(0, job.targets, job.k_lo, job.k_hi)
    np.testing.assert_array_equal(nb, nref)
    ok = nref > 0
    assert ok.sum() >= 8
    rel = np.abs(got[ok] - ref[ok]) / np.abs(ref[ok])
    _say("max rel err per bin", rel.max())
    assert rel.max() <= tol


def test_invalid_tables_refused():
    job = _job(32)
    with P.Plan(32, prec="f64") as pl:
        pl.generate_field(0, 3, job.spectrum, job.ngmap)
        om0, _ = pl.spectrum(0, job.targets, job.k_lo, job.k_hi)
        s, phi, e = P.sigw_kernel_table(pl.desc, 0)
        bad_e = e.copy()
        bad_e[5] = bad_e[4]
        bad_s = s.copy()
        bad_s[2] = np.nan
        for args in ((0, s, phi, bad_e), (1, bad_s, phi, None), (2, s, phi, None)):
            with pytest.raises(_lib.SigwError):
                pl.set_kernel_table(*args)
        om1, _ = pl.spectrum(0, job.targets, job.k_lo, job.k_hi)
    np.testing.assert_array_equal(om0.view(np.uint64), om1.view(np.uint64))


@pytest.fixture(scope="module")
def tabs_w06():
    return eos.tables_w(0.6)


@pytest.mark.parametrize("N,prec,tol", [(32, "f64", 1e-10), (64, "f32", 1e-4)])
def test_constant_w_tables_vs_oracle(N, prec, tol, tabs_w06):
    job = _job(N)
    ph = field.phi_hat(N, job.L, 5, job.spectrum, job.ngmap)
    _say(f"constant-w (0.6) tables N={N} prec={prec}")
    ref, nref = spectrum.omega_spectrum(ph, tabs_w06[0], tabs_w06[1], job.targets, job.k_lo, job.k_hi, job.L)
    ok = nref > 0
    assert ok.sum() >= 8
    with P.Plan(N, prec=prec) as pl:
        pl.generate_field(0, 5, job.spectrum, job.ngmap)
        for m in range(2):
            pl.set_kernel_table(m, tabs_w06[m].sigma, tabs_w06[m].phi, tabs_w06[m].edges)
        got, nb = pl.spectrum(0, job.targets, job.k_lo, job.k_hi)
        np.testing.assert_array_equal(nb, nref)
        rel = np.abs(got[ok] - ref[ok]) / np.abs(ref[ok])
        _say("  oracle tables: max rel err per bin", rel.max())
        assert rel.max() <= tol
        pl.set_equation_of_state(0.6)          # the library's own builder
        got2, nb2 = pl.spectrum(0, job.targets, job.k_lo, job.k_hi)
    np.testing.assert_array_equal(nb2, nref)
    rel2 = np.abs(got2[ok] - ref[ok]) / np.abs(ref[ok])
    _say("  library tables: max rel err per bin", rel2.max())
    assert rel2.max() <= max(tol, 1e-6)
