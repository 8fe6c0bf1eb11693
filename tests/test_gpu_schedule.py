"""The x-pass schedules and their autotuner, through the C ABI.

Every compiled schedule of the fused inverse-x / products / forward-x
kernel (z chunk per workgroup, occupancy target) computes the same values
in the same order, so spectra must be bit-for-bit identical across
schedules; the default one is held to the FP64 oracle at 64^3 (FP32: 1e-4
per bin, FP64: 1e-10).  The autotuner must pick one of the compiled
schedules, and later plans of the same size created with autotune=1 must
reuse its choice.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import decomposition, field, spectrum

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2605_27231_amd")
from paper_2605_27231_amd import _lib  # noqa: E402


def _say(*a):
    print(*a, flush=True)


def _job64():
    N, L = 64, 2 * math.pi
    e, t = W.log_bins(N, L, 16)
    lo, hi = W.shells_from_edges(e)
    return W.Job(N=N, L=L, spectrum=W.Lognormal(1e-2, 0.5, 8.0), ngmap=W.NGMap("local", F_NL=3.0),
                 k_lo=lo, k_hi=hi, targets=t)


@pytest.fixture(scope="module")
def oracle64():
    job = _job64()
    tabs = decomposition.tables()
    ph = field.phi_hat(job.N, job.L, 5, job.spectrum, job.ngmap)
    return spectrum.omega_spectrum(ph, tabs[0], tabs[1], job.targets, job.k_lo, job.k_hi, job.L)


def _all_schedules(pl, slot, job):
    idx0, count, _ = pl.schedule()
    assert idx0 == 0 and count >= 1
    out = []
    for i in range(count):
        pl.set_schedule(i)
        _say(f"  schedule {i}: {pl.schedule()[2]}")
        out.append(pl.spectrum(slot, job.targets, job.k_lo, job.k_hi))
    return out, count


@pytest.mark.parametrize("prec,tol", [("f32", 1e-4), ("f64", 1e-10)])
def test_schedules_bit_identical_64(oracle64, prec, tol):
    job = _job64()
    ref, nref = oracle64
    _say(f"schedules 64^3 {prec}")
    with P.Plan(job.N, prec=prec) as pl:
        pl.generate_field(0, 5, job.spectrum, job.ngmap)
        res, count = _all_schedules(pl, 0, job)
    assert count == 3
    om0, nb0 = res[0]
    np.testing.assert_array_equal(nb0, nref)
    ok = nref > 0
    rel = np.abs(om0[ok] - ref[ok]) / np.abs(ref[ok])
    assert rel.max() <= tol, rel.max()
    for om, nb in res[1:]:
        np.testing.assert_array_equal(nb, nb0)
        np.testing.assert_array_equal(om.view(np.uint64), om0.view(np.uint64))


def test_schedules_bit_identical_256():
    job = W.config_local_ng(256, 64)
    b = int(np.argmin(np.abs(job.targets - job.spectrum.k_star * 2 / math.sqrt(3))))
    sub = W.Job(N=job.N, L=job.L, spectrum=job.spectrum, ngmap=job.ngmap, k_lo=job.k_lo[b - 1:b + 2],
                k_hi=job.k_hi[b - 1:b + 2], targets=job.targets[b - 1:b + 2])
    _say("schedules 256^3 f32, 3 targets at the peak")
    with P.Plan(256, prec="f32") as pl:
        pl.generate_field(0, 1, job.spectrum, job.ngmap)
        res, count = _all_schedules(pl, 0, sub)
    assert count >= 2
    for om, nb in res[1:]:
        np.testing.assert_array_equal(nb, res[0][1])
        np.testing.assert_array_equal(om.view(np.uint64), res[0][0].view(np.uint64))


def test_schedules_bit_identical_384_and_repeatable():
    """At 384^3 the x pass hands off LDS between its phases with barriers
    that leave the next tile's loads in flight: every schedule must still
    give the same bits, and the same schedule the same bits twice."""
    job = W.config_local_ng(256, 64)
    L = job.L
    targets = np.array([15.0, 23.0, 40.0])
    lo, hi = targets - 0.5, targets + 0.5
    sub = W.Job(N=384, L=L, spectrum=job.spectrum, ngmap=job.ngmap, k_lo=lo, k_hi=hi, targets=targets)
    _say("schedules 384^3 f32, 3 targets")
    with P.Plan(384, L=L, prec="f32") as pl:
        pl.generate_field(0, 2, job.spectrum, job.ngmap)
        res, count = _all_schedules(pl, 0, sub)
        pl.set_schedule(0)
        again = pl.spectrum(0, sub.targets, sub.k_lo, sub.k_hi)
    assert count >= 2
    np.testing.assert_array_equal(again[0].view(np.uint64), res[0][0].view(np.uint64))
    for om, nb in res[1:]:
        np.testing.assert_array_equal(nb, res[0][1])
        np.testing.assert_array_equal(om.view(np.uint64), res[0][0].view(np.uint64))
    assert np.all(res[0][1] > 0)


def test_autotune_choice_and_reuse():
    job = _job64()
    _say("autotune 128^3 f32")
    with P.Plan(128, prec="f32") as pl:
        text = pl.autotune(force=True)
        idx, count, text2 = pl.schedule()
        _say("  ", text)
        assert text == text2 and text.startswith("tzx=") and "timed over" in text
        assert 0 <= idx < count and count == 3
        pl.generate_field(0, 2, job.spectrum, job.ngmap)
        tuned = pl.spectrum(0, job.targets * 2, job.k_lo * 2, job.k_hi * 2)
        pl.set_schedule(0)
        dflt = pl.spectrum(0, job.targets * 2, job.k_lo * 2, job.k_hi * 2)
        with pytest.raises(_lib.SigwError):
            pl.set_schedule(count)
    np.testing.assert_array_equal(tuned[0].view(np.uint64), dflt[0].view(np.uint64))
    # a later plan of the same size reuses the process-wide choice without timing again
    with P.Plan(128, prec="f32", autotune=1) as pl2:
        idx2, _, text3 = pl2.schedule()
    assert idx2 == idx and text3 == text
    # a size that was never tuned starts from the default and tunes at creation
    with P.Plan(32, prec="f32", autotune=1) as pl3:
        idx3, count3, text4 = pl3.schedule()
    assert count3 == 1 and idx3 == 0 and text4.startswith("tzx=8 occ=3")
