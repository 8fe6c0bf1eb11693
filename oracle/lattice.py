"""Mode grids and the continuum Fourier convention on the periodic lattice.

Convention (Sec. III, the two-point function, and Sec. IV, the real-space
auxiliary fields): for a box of side L with N sites per side, spacing L/N,
cell volume dV = (L/N)^3 and volume V = L^3,

    X_hat(n) = dV * sum_x X(x) exp(-i q_n . x)        (forward, "DFT times dV")
    X(x)     = (1/V) * sum_n exp(+i q_n . x) X_hat(n)  (inverse)

with q_n = k_F n, k_F = 2 pi / L and n the signed integer representative in
[-N/2, N/2).  Real fields keep the half spectrum with the *first* axis halved:
index kx = 0..N/2 (kx = N/2 is the Nyquist plane, signed value -N/2), full
ky and kz.  That is exactly ``numpy.fft.fftn(X)[:N//2+1]``.
"""
from __future__ import annotations

import math
import os

import numpy as np
import scipy.fft as sfft

def _threads() -> int:
    """Host threads for the FFT library: the CPUs this process may run on,
    capped by OMP_NUM_THREADS when that is set."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return max(1, n)


_WORKERS = _threads()
_AXES = (1, 2, 0)   # transform order; the last axis listed (x) is the halved one


def kf(L: float) -> float:
    return 2.0 * math.pi / L


def signed_full(N: int) -> np.ndarray:
    """Signed integer representatives of the DFT indices 0..N-1."""
    return np.fft.fftfreq(N, d=1.0 / N).round().astype(np.int64)


def signed_half(N: int) -> np.ndarray:
    """Signed representatives of the halved axis indices 0..N/2."""
    return signed_full(N)[: N // 2 + 1] if N > 1 else np.zeros(1, np.int64)


def half_shape(N: int):
    return (N // 2 + 1, N, N)


def mode_grids_half(N: int):
    """(nx, ny, nz) broadcastable integer grids on the half-spectrum layout."""
    nx = signed_half(N)
    nx = nx.copy()
    nx[-1] = -(N // 2)
    ny = signed_full(N)
    nz = signed_full(N)
    return nx[:, None, None], ny[None, :, None], nz[None, None, :]


def mode_grids_full(N: int):
    n = signed_full(N)
    return n[:, None, None], n[None, :, None], n[None, None, :]


def n2_half(N: int) -> np.ndarray:
    nx, ny, nz = mode_grids_half(N)
    return (nx * nx + ny * ny + nz * nz).astype(np.int64)


def qtilde_half(N: int, L: float):
    """Gradient wavevector components k_F n_j, set to zero where n_j = -N/2
    (the Nyquist index has no sign, so the derivative there is taken as zero;
    this keeps i*q*X Hermitian for a real X)."""
    nx, ny, nz = mode_grids_half(N)
    k = kf(L)
    out = []
    for n in (nx, ny, nz):
        q = (k * n).astype(np.float64)
        q = np.where(n == -(N // 2), 0.0, q)
        out.append(q)
    return out


def forward(X: np.ndarray, L: float) -> np.ndarray:
    """X_hat = dV * DFT(X) for a real N^3 field, on the half layout."""
    N = X.shape[0]
    dV = (L / N) ** 3
    return dV * sfft.rfftn(X, axes=_AXES, workers=_WORKERS)


def inverse(Xh: np.ndarray, L: float) -> np.ndarray:
    """X(x) = (1/V) sum_n exp(i q.x) X_hat(n) for a Hermitian half spectrum."""
    N = Xh.shape[1]
    V = L ** 3
    return (N ** 3 / V) * sfft.irfftn(Xh, s=(N, N, N), axes=_AXES, workers=_WORKERS)


def dft_plain(X: np.ndarray) -> np.ndarray:
    """Un-normalised DFT sum_x X(x) exp(-2 pi i n.x/N) on the half layout."""
    return sfft.rfftn(X, axes=_AXES, workers=_WORKERS)


def half_weights(N: int) -> np.ndarray:
    """How many full-grid modes each half-layout mode stands for: the planes
    kx = 0 and kx = N/2 contain both n and -n, every other plane stands for
    its mirror too."""
    w = np.full(N // 2 + 1, 2, dtype=np.int64)
    w[0] = 1
    w[-1] = 1
    return w[:, None, None] * np.ones((1, N, N), dtype=np.int64)
