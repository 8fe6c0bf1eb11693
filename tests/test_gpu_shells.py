"""Shells that hold no lattice mode, and shell edges at the extremes (Sec. IV
shell estimator), through the C ABI.

* A shell whose only integer |n|^2 is 7 (not a sum of three squares) holds
  no mode: N_b = 0, Omega = 0, and no per-target kernel is launched; next to
  ordinary shells it changes neither their results nor their launch count.
* A negative k_lo counts the same modes as k_lo = 0, and an upper edge far
  beyond the lattice (1e12) the same as one just above the corner mode.
"""
import math

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2605_27231_amd")

HOT = ("gen_z", "ypass", "xprod", "zbin")


def _launches(pl):
    return {k: pl.kernel_time(k)[1] for k in HOT}


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_shell_without_modes_launches_nothing(prec):
    N, L = 16, 2 * math.pi
    job = W.config_plain_fp64(N)
    k7 = math.sqrt(7.0)
    print(f"phantom shell |n|^2 = 7, {prec}", flush=True)
    with P.Plan(N, L=L, prec=prec) as pl:
        pl.generate_field(0, 0, job.spectrum, job.ngmap)
        pl.set_timing(True)
        om, nb = pl.spectrum(0, [k7], [k7 - 0.01], [k7 + 0.01])
        assert nb[0] == 0 and om[0] == 0.0
        assert _launches(pl) == {k: 0 for k in HOT}
        # ordinary shells alone, then with the empty one between them
        t = np.array([3.0, 5.0])
        pl.set_timing(True)
        om_a, nb_a = pl.spectrum(0, t, t - 0.5, t + 0.5)
        alone = _launches(pl)
        pl.set_timing(True)
        om_b, nb_b = pl.spectrum(0, [3.0, k7, 5.0], [2.5, k7 - 0.01, 4.5], [3.5, k7 + 0.01, 5.5])
        assert _launches(pl) == alone
        np.testing.assert_array_equal(om_b[[0, 2]], om_a)
        np.testing.assert_array_equal(nb_b[[0, 2]], nb_a)
        assert nb_b[1] == 0 and om_b[1] == 0.0
        pl.set_timing(False)


def test_extreme_shell_edges():
    N, L = 16, 2 * math.pi
    job = W.config_plain_fp64(N)
    corner = math.sqrt(3.0) * N / 2          # k_F |n| of the corner mode, k_F = 1
    print("shell edges: negative k_lo, k_hi = 1e12", flush=True)
    with P.Plan(N, L=L, prec="f64") as pl:
        pl.generate_field(0, 0, job.spectrum, job.ngmap)
        _, nb_neg = pl.spectrum(0, [3.0], [-5.0], [3.0])
        _, nb_zero = pl.spectrum(0, [3.0], [0.0], [3.0])
        assert nb_neg[0] == nb_zero[0] > 0
        om_big, nb_big = pl.spectrum(0, [20.0], [12.0], [1e12])
        om_cor, nb_cor = pl.spectrum(0, [20.0], [12.0], [corner + 1e-6])
        assert nb_big[0] == nb_cor[0] > 0
        assert om_big[0] == om_cor[0]
