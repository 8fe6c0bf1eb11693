"""The per-target box protocol through the C ABI against the oracle
(oracle/adaptive.py): the box side per target, N_b, and Omega (FP64 path
1e-10 relative, FP32 path 1e-4).  The slot is left empty afterwards, the
plan's own box is unchanged, and a bad eps is refused."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import adaptive, decomposition, spectrum

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2605_27231_amd")
from paper_2605_27231_amd import _lib  # noqa: E402


@pytest.mark.parametrize("N,prec,tol", [(32, "f64", 1e-10), (64, "f32", 1e-4)])
def test_adaptive_matches_oracle(N, prec, tol):
    spec = W.Lognormal(1e-2, 0.5, 8.0)
    ngmap = W.NGMap("local", F_NL=1.5)
    ks = np.array([4.0, 9.0, 15.0, 20.0])      # k_bar = 15.2: the last target sets its own box
    print(f"adaptive N={N} {prec}", flush=True)
    ref = adaptive.omega_adaptive(N, 6, spec, ngmap, ks, 0.1, tabs=decomposition.tables())
    with P.Plan(N, prec=prec) as pl:
        om, nb, box = pl.spectrum_adaptive(0, 6, spec, ngmap, ks, 0.1)
        with pytest.raises(_lib.SigwError) as e:             # the slot was left empty
            pl.spectrum(0, [2.0], [1.5], [2.5])
        assert e.value.status == _lib.SIGW_E_STATE
        with pytest.raises(_lib.SigwError):
            pl.spectrum_adaptive(0, 6, spec, ngmap, ks, 1.5)
        # the plan's own box is back: a field generated now matches the 2 pi box
        pl.generate_field(0, 6, spec, ngmap)
        om2, nb2 = pl.spectrum(0, [5.0], [4.5], [5.5])
    for b, (o, n, L) in enumerate(ref):
        assert abs(box[b] - L) <= 1e-12 * L
        assert nb[b] == n
        assert abs(om[b] - o) <= tol * o, (b, om[b], o)
        print(f"  k={ks[b]} L={L:.4f} Omega={o:.4e}", flush=True)
    assert nb2[0] == spectrum.mode_counts(N, 2 * math.pi, [4.5], [5.5])[0] and om2[0] > 0
