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
    """At k = k_F the support is the ball |n| <= 15 and the shell |n| = 1:
    the target runs on a 32^3 grid (2 Rc + Kc + 1 = 32), where gen_z writes
    only the ball's rows and xprod reads only the planes kx <= 15."""
    N, L, cb, na = 64, 2 * math.pi, 8, 50
    assert bench.target_grid(N, L, 1.0, 15.0, 1) == 32
    ab = bench.algorithmic_bytes(N, L, cb, na, 15.0, [1.0], [0.5], [1.5])
    M = 32
    ky = np.fft.fftfreq(M, 1.0 / M)
    rows = int(((np.arange(16)[:, None] ** 2 + ky[None, :] ** 2) <= 226).sum())
    assert ab["gen_z"] == (rows * M + 2 * na * rows * M) * cb
    assert ab["xprod"] == (3 * na * 16 * M * M + 6 * 2 * M * M) * cb


@pytest.mark.parametrize("N,rc,kc", [(32, 5, 3), (32, 3, 7), (64, 9, 4)])
def test_coarse_grid_reproduces_shell(N, rc, kc):
    """Products of fields supported on |n_c| <= rc, transformed on the N grid
    and on the smallest M with M > 2 rc + kc and M > 2 kc + 1, agree on
    every mode of the shell |n_c| <= kc (continuum normalisation, as the hot
    path uses): no product mode aliases onto the shell on either grid."""
    L = 2 * math.pi
    M = next(m for m in bench.GRID_SIZES if m >= max(2 * rc + kc + 1, 2 * kc + 2))
    assert M < N
    rng = np.random.default_rng(N + rc + kc)
    n = np.fft.fftfreq(N, 1.0 / N).astype(int)
    box = (np.abs(n)[:, None, None] <= rc) & (np.abs(n)[None, :, None] <= rc) & (np.abs(n)[None, None, :] <= rc)
    fields = []
    for _ in range(2):
        a = (rng.standard_normal((N, N, N)) + 1j * rng.standard_normal((N, N, N))) * box
        a = 0.5 * (a + np.conj(a[(-n)[:, None, None] % N, (-n)[None, :, None] % N, (-n)[None, None, :] % N]))
        fields.append(a)                                  # Hermitian: real fields
    def on_grid(G):
        m = np.fft.fftfreq(G, 1.0 / G).astype(int)
        idx = np.ix_(m % N, m % N, m % N)
        dV = (L / G) ** 3
        x = [np.fft.ifftn(f[idx]) * G ** 3 / L ** 3 for f in fields]      # (1/V) sum e^{iqx} f
        return dV * np.fft.fftn((x[0] * x[1]).real), m
    QN, mN = on_grid(N)
    QM, mM = on_grid(M)
    shell = [(a, b, c) for a in range(-kc, kc + 1) for b in range(-kc, kc + 1) for c in range(-kc, kc + 1)]
    vN = np.array([QN[a % N, b % N, c % N] for a, b, c in shell])
    vM = np.array([QM[a % M, b % M, c % M] for a, b, c in shell])
    assert np.max(np.abs(vN - vM)) <= 1e-12 * np.max(np.abs(vN))
    # one grid size too small does alias (M - 1 would allow it): the bound is needed
    if 2 * rc + kc + 1 > 8 and M // 2 >= 2 * kc + 2 and M // 2 in bench.GRID_SIZES:
        Qs, _ = on_grid(M // 2)
        vs = np.array([Qs[a % (M // 2), b % (M // 2), c % (M // 2)] for a, b, c in shell])
        assert np.max(np.abs(vN - vs)) > 1e-6 * np.max(np.abs(vN))
