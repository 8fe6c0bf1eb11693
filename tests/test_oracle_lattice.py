"""Pins of the lattice Fourier convention (P7).

* forward/inverse against the explicit sums  dV sum_x exp(-i q.x) X(x)  and
  (1/V) sum_n exp(i q.x) X_hat(n)  written out on 4^3, 6^3 and 8^3 lattices;
* Parseval: sum_x |X|^2 dV = (1/V) sum_n |X_hat|^2 (with half-layout weights);
* the half layout is numpy.fft.fftn(X)[:N/2+1] and is Hermitian;
* the gradient wavevector is zero at the Nyquist index and odd elsewhere.
"""
import itertools
import math

import numpy as np
import pytest

from oracle import lattice


def _explicit_forward(X, L):
    N = X.shape[0]
    dV = (L / N) ** 3
    k = 2 * math.pi / L
    n = lattice.signed_full(N)
    x = np.arange(N) * (L / N)
    out = np.zeros((N // 2 + 1, N, N), dtype=np.complex128)
    for a, b, c in itertools.product(range(N // 2 + 1), range(N), range(N)):
        ph = np.exp(-1j * k * (n[a] * x[:, None, None] + n[b] * x[None, :, None] + n[c] * x[None, None, :]))
        out[a, b, c] = dV * np.sum(X * ph)
    return out


@pytest.mark.parametrize("N", [4, 6, 8])
def test_forward_matches_explicit_sum(N):
    L = 3.7
    X = np.random.default_rng(N).standard_normal((N, N, N))
    np.testing.assert_allclose(lattice.forward(X, L), _explicit_forward(X, L), rtol=0, atol=1e-12)


@pytest.mark.parametrize("N", [4, 6])
def test_inverse_matches_explicit_sum(N):
    L = 2.3
    X = np.random.default_rng(N + 10).standard_normal((N, N, N))
    Xh = lattice.forward(X, L)
    # explicit inverse over the full grid, rebuilt from the half layout
    full = np.fft.fftn(X) * (L / N) ** 3
    np.testing.assert_allclose(full[: N // 2 + 1], Xh, atol=1e-12)
    V = L ** 3
    k = 2 * math.pi / L
    n = lattice.signed_full(N)
    x = np.arange(N) * (L / N)
    Y = np.zeros((N, N, N))
    for a, b, c in itertools.product(range(N), repeat=3):
        ph = np.exp(1j * k * (n[a] * x[:, None, None] + n[b] * x[None, :, None] + n[c] * x[None, None, :]))
        Y += np.real(full[a, b, c] * ph) / V
    np.testing.assert_allclose(lattice.inverse(Xh, L), Y, atol=1e-12)
    np.testing.assert_allclose(Y, X, atol=1e-12)


def test_parseval_and_hermitian_planes():
    N, L = 16, 5.0
    X = np.random.default_rng(2).standard_normal((N, N, N))
    Xh = lattice.forward(X, L)
    dV, V = (L / N) ** 3, L ** 3
    lhs = np.sum(X * X) * dV
    rhs = np.sum(lattice.half_weights(N) * np.abs(Xh) ** 2) / V
    assert lhs == pytest.approx(rhs, rel=1e-13)
    # the kx = 0 and kx = N/2 planes hold X(-n) = X(n)*
    for a in (0, N // 2):
        P = Xh[a]
        Pm = P[(-np.arange(N)) % N][:, (-np.arange(N)) % N]
        np.testing.assert_allclose(P, np.conj(Pm), atol=1e-12)


def test_gradient_wavevector():
    N, L = 8, 2 * math.pi
    qx, qy, qz = lattice.qtilde_half(N, L)
    assert qx.shape == (N // 2 + 1, 1, 1) and qy.shape == (1, N, 1)
    assert qx[-1, 0, 0] == 0.0 and qy[0, N // 2, 0] == 0.0 and qz[0, 0, N // 2] == 0.0
    assert qy[0, 1, 0] == 1.0 and qy[0, N - 1, 0] == -1.0
    assert lattice.n2_half(N)[N // 2, 0, 0] == (N // 2) ** 2
