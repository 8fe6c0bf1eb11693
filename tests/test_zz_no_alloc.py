"""The allocation-free spectrum (sigw_spectrum_noalloc, for callers that
cannot allocate device memory) against the plan-based sigw_spectrum, through
the C ABI, on two calls in a row, the second on a smaller lattice: FP64 within
1e-10 relative per bin, FP32 within 1e-4, mode counts exact.  The shells
include ones that run on smaller grids, one at the Nyquist corner and one
that holds no lattice mode."""
import math

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2605_27231_amd")
from paper_2605_27231_amd import api  # noqa: E402


def _case(N, prec):
    L = 2 * math.pi
    spec = W.Lognormal(1e-2, 0.5, N / 8.0)
    ngmap = W.NGMap("local", F_NL=3.0)
    e, t = W.linear_bins(N, L, N // 2)
    lo, hi = W.shells_from_edges(e)
    k7 = math.sqrt(7.0)
    t = np.append(t, [k7, math.sqrt(3.0) * N / 2 - 0.25])
    lo = np.append(lo, [k7 - 0.01, math.sqrt(3.0) * N / 2 - 0.5])
    hi = np.append(hi, [k7 + 0.01, 1e9])
    with P.Plan(N, L=L, prec=prec) as pl:
        pl.generate_field(0, 11, spec, ngmap)
        phi = pl.get_phi_hat(0)
        om_ref, nb_ref = pl.spectrum(0, t, lo, hi)
    return phi, t, lo, hi, om_ref, nb_ref


@pytest.mark.parametrize("prec,tol", [("f64", 1e-10), ("f32", 1e-4)])
def test_noalloc_equals_plan_path_two_calls(prec, tol):
    for N in (64, 32):          # the second call on a smaller input
        print(f"no-alloc spectrum N={N} {prec}", flush=True)
        phi, t, lo, hi, om_ref, nb_ref = _case(N, prec)
        om, nb = api.sigw_spectrum_noalloc(P.plan_desc(N, prec=prec), phi, t, lo, hi)
        np.testing.assert_array_equal(nb, nb_ref)
        ok = nb_ref > 0
        assert ok.sum() >= N // 2 - 2 and not ok[-2]
        rel = np.abs(om[ok] - om_ref[ok]) / np.abs(om_ref[ok])
        print(f"  max rel err {rel.max():.2e} over {ok.sum()} shells", flush=True)
        assert rel.max() <= tol
        assert np.all(om[~ok] == 0.0)
