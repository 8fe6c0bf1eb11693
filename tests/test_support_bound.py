"""The weighted fields phi_a(|q|/k) Phi_hat vanish outside |q| < u_max k
(u_max the last edge of the u grid, Sec. V), which is what lets the hot path
skip the rows and planes outside that ball.  These checks pin the bound that
the benchmark's byte accounting uses (the library prunes with the same
formula) against the oracle's own interval lookup: every mode the oracle
weights lies inside it, and it is tight to one |n|^2 step."""
import math

import numpy as np
import pytest

import bench
from oracle import decomposition, lattice, spectrum


@pytest.fixture(scope="module")
def table():
    return decomposition.tables()[0]


@pytest.mark.parametrize("N", [16, 32, 64])
@pytest.mark.parametrize("k_b", [0.3, 1.0, 1.7, 2.9, 5.0])
def test_oracle_support_inside_bound(table, N, k_b):
    L = 2 * math.pi
    idx = spectrum.interval_lookup(N, L, k_b, table)
    n2 = lattice.n2_half(N)
    bound = bench.support_n2(N, L, k_b, float(table.edges[-1]))
    live = n2[idx >= 0]
    assert live.size > 0
    assert live.max() <= bound
    if bound < 3 * (N // 2) ** 2:
        # no mode between the last weighted one and the bound but the margin
        r = float(table.edges[-1]) * k_b / lattice.kf(L)
        assert bound <= r * r + 2


def test_pruned_byte_model_reduces_to_full_at_large_k():
    """Above k = sqrt(3) (N/2) k_F / u_max the ball covers the cube and the
    per-launch bytes equal the unpruned counts."""
    N, L, cb, na = 32, 2 * math.pi, 8, 50
    k = 3.0 * (N // 2) / 15.0 * 2
    ab = bench.algorithmic_bytes(N, L, cb, na, 15.0, [k], [k - 0.5], [k + 0.5])
    H = N // 2 + 1
    FS = H * N * N
    st = bench.stage_terms(N, cb, na)
    assert st == na
    assert ab["gen_z"] == (FS + 2 * st * FS) * cb
    assert ab["ypass"] == 5 * st * FS * cb
    n2_hi = bench.shell_n2_hi(N, L, k - 0.5, k + 0.5)
    n_planes = min(H - 1, math.isqrt(n2_hi)) + 1
    assert ab["xprod"] == (3 * na * FS + 6 * n_planes * N * N) * cb


def test_pruned_byte_model_small_k():
    """At k = k_F the support is the ball |n| <= 15: gen_z writes only its
    rows and xprod reads only the planes kx <= 15."""
    N, L, cb, na = 64, 2 * math.pi, 8, 50
    ab = bench.algorithmic_bytes(N, L, cb, na, 15.0, [1.0], [0.5], [1.5])
    ky = np.fft.fftfreq(N, 1.0 / N)
    rows = int(((np.arange(16)[:, None] ** 2 + ky[None, :] ** 2) <= 226).sum())
    assert ab["gen_z"] == (rows * N + 2 * na * rows * N) * cb
    assert ab["xprod"] == (3 * na * 16 * N * N + 6 * 2 * N * N) * cb
