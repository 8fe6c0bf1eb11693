"""Jackknife error of the shell estimator (Sec. IV, the jackknife equations).

The paper transforms the shell's field to real space, splits the box into
M^3 sub-volumes and forms M^3 replica measurements, each leaving one
sub-volume out; the error is sigma^2 = (M^3 - 1)/M^3 sum_i (P^(i) - mean)^2.
Reading R24 (the paper leaves the replica estimator implicit): for each
kernel m the TT projection of the shell's modes,
    Y^(m)(n) = Lambda(X^(m)(n)) = P X P - 1/2 P tr(P X P)   (n in the shell, 0 elsewhere),
is transformed to real space, h^(m)_ij(x) = (1/V) sum_n exp(i q.x) Y^(m)_ij(n)
(real, since X is Hermitian; the shell must lie below the Nyquist frequency
so that the projector is even in n).  By Parseval the shell power
S_b = sum_n sum_m |Y^(m)(n)|^2 (the quantity of the shell estimator, since
|Lambda X|^2 = sum_ij |P X P|^2 - 1/2 |tr P X P|^2) splits over sub-volumes:
    S_i = (V^2 / N^3) sum_{x in sub-volume i} sum_m sum_ij |h^(m)_ij(x)|^2,  sum_i S_i = S_b.
Replica i: S^(i) = M^3/(M^3 - 1) (S_b - S_i), Omega^(i) from S^(i) and N_b
as for the full shell; the reported error is the jackknife sigma of Omega.

Test infrastructure only: nothing on the product path imports this.
"""
from __future__ import annotations

import numpy as np

from . import lattice
from .spectrum import PAIRS, omega_from_sum, shell_mask


def tt_project(X: np.ndarray, khat: np.ndarray) -> np.ndarray:
    """Lambda(X) = P X P - 1/2 P tr(P X P) for (M, 3, 3) tensors and unit vectors."""
    P = np.eye(3)[None, :, :] - khat[:, :, None] * khat[:, None, :]
    Y = P @ X @ P
    tr = np.trace(Y, axis1=1, axis2=2)
    return Y - 0.5 * P * tr[:, None, None]


def shell_tt_fields(Qs: np.ndarray, Qc: np.ndarray, k_b: float, lo: float, hi: float, L: float) -> np.ndarray:
    """Real-space fields h^(m)_ij, shape (2, 3, 3, N, N, N)."""
    N = Qs.shape[2]
    if hi > lattice.kf(L) * (N // 2):
        raise ValueError("the jackknife needs the shell below the Nyquist frequency")
    mask = shell_mask(N, L, lo, hi)
    nx, ny, nz = lattice.mode_grids_half(N)
    n = np.stack(np.broadcast_arrays(nx, ny, nz), axis=-1)[mask].astype(np.float64)
    khat = n / np.linalg.norm(n, axis=1)[:, None]
    pref = 4.0 / (k_b * k_b)
    out = np.zeros((2, 3, 3, N, N, N))
    for m, (Qh, sign) in enumerate(((Qs, -1.0), (Qc, +1.0))):
        X = np.empty((int(mask.sum()), 3, 3), dtype=np.complex128)
        for c, (i, j) in enumerate(PAIRS):
            X[:, i, j] = sign * pref * Qh[c][mask]
            X[:, j, i] = X[:, i, j]
        Y = tt_project(X, khat)
        for i in range(3):
            for j in range(3):
                full = np.zeros((N // 2 + 1, N, N), dtype=np.complex128)
                full[mask] = Y[:, i, j]
                out[m, i, j] = lattice.inverse(full, L)
    return out


def subvolume_sums(h: np.ndarray, L: float, M: int) -> np.ndarray:
    """S_i for the M^3 sub-volumes (i = (a M + b) M + c for the block at
    x in [a, a+1) N/M, y in [b, b+1) N/M, z in [c, c+1) N/M)."""
    N = h.shape[-1]
    if M < 2 or N % M:
        raise ValueError("M must be >= 2 and divide N")
    V = L ** 3
    e = np.sum(h * h, axis=(0, 1, 2))                        # sum_m sum_ij |h|^2 per site
    B = N // M
    S = e.reshape(M, B, M, B, M, B).sum(axis=(1, 3, 5))
    return (V * V / N ** 3) * S.reshape(-1)


def jackknife_from_sums(S_i: np.ndarray, N_b: int, k_b: float, L: float):
    """(Omega of the full shell, sigma, replica Omegas)."""
    M3 = len(S_i)
    S = float(np.sum(S_i))
    rep = np.array([omega_from_sum(M3 / (M3 - 1) * (S - s), N_b, k_b, L) for s in S_i])
    mean = float(np.mean(rep))
    sigma = float(np.sqrt((M3 - 1) / M3 * np.sum((rep - mean) ** 2)))
    return omega_from_sum(S, N_b, k_b, L), sigma, rep
