"""Per-target convolution engine, TT projection and shell average (Sec. III, IV).

For one target wavenumber k_b and one kernel m in {s, c} (Eq. final_envelopes):

    u(n)          = k_F sqrt(|n|^2) / k_b                (evaluated in this order)
    V_a(n)        = phi_a(u(n)) Phi_hat(n)                (auxiliary fields, Sec. IV)
    G_a,j(x)      = (1/V) sum_n exp(i q.x) i q_j V_a(n)   (gradients d_j V_a)
    Q_ij(x)       = sum_a sigma_a G_a,i(x) G_a,j(x)
    Q_hat_ij(n)   = dV DFT(Q_ij)(n)
    X^(s) = -(4/k_b^2) Q_hat^(s),  X^(c) = +(4/k_b^2) Q_hat^(c)

and A_lambda = e^lambda_ij X^(s)_ij, B_lambda = e^lambda_ij X^(c)_ij.  The sum
over the two polarisations of |e^lambda : X|^2 equals X* : Lambda : X with the
TT projector Lambda_ij,lm = 1/2 (P_il P_jm + P_im P_jl - P_ij P_lm),
P = 1 - k-hat k-hat^T; for a symmetric X this is
sum_ij |Y_ij|^2 - 1/2 |tr Y|^2 with Y = P X P.

Shell average (Sec. IV):  P_X(k_b) = 1/(V N_b) sum_{n in shell} |X_n|^2, over
all n != 0 with k_F |n| in [lo_b, hi_b); every mode in the shell is evaluated
with the target k_b.  Omega^(RD)(k_b) = k_b^3/(48 pi^2) sum_lambda (P_A + P_B)
(Sec. III).
"""
from __future__ import annotations

import math

import numpy as np

from . import lattice

PAIRS = ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))


def interval_lookup(N: int, L: float, k_b: float, table):
    """Interval index of u(n) = k_F sqrt(n^2) / k_b for every half-layout mode."""
    n2 = lattice.n2_half(N).astype(np.float64)
    u = lattice.kf(L) * np.sqrt(n2) / k_b
    return table.interval_index(u)


def source_qhat(phi_hat: np.ndarray, table, k_b: float, L: float) -> np.ndarray:
    """Q_hat^(m)_ij for one kernel table, as a (6, N/2+1, N, N) complex array in
    the component order xx, yy, zz, xy, xz, yz."""
    N = phi_hat.shape[1]
    idx = interval_lookup(N, L, k_b, table)
    valid = idx >= 0
    safe = np.where(valid, idx, 0)
    qt = lattice.qtilde_half(N, L)
    Q = np.zeros((6, N, N, N), dtype=np.float64)
    for a in range(len(table.sigma)):
        phi_a = np.where(valid, table.phi[safe, a], 0.0)
        V = phi_a * phi_hat
        G = [lattice.inverse(1j * qt[j] * V, L) for j in range(3)]
        s = table.sigma[a]
        for c, (i, j) in enumerate(PAIRS):
            Q[c] += s * (G[i] * G[j])
    return np.stack([lattice.forward(Q[c], L) for c in range(6)])


def sym3(Qh_modes: np.ndarray) -> np.ndarray:
    """(6, M) components -> (M, 3, 3) symmetric matrices."""
    M = Qh_modes.shape[1]
    X = np.empty((M, 3, 3), dtype=np.complex128)
    for c, (i, j) in enumerate(PAIRS):
        X[:, i, j] = Qh_modes[c]
        X[:, j, i] = Qh_modes[c]
    return X


def tt_power(X: np.ndarray, khat: np.ndarray) -> np.ndarray:
    """sum_lambda |e^lambda : X|^2 = sum_ij |Y_ij|^2 - |tr Y|^2 / 2, Y = P X P."""
    P = np.eye(3)[None, :, :] - khat[:, :, None] * khat[:, None, :]
    Y = P @ X @ P
    tr = np.trace(Y, axis1=1, axis2=2)
    return np.sum(np.abs(Y) ** 2, axis=(1, 2)) - 0.5 * np.abs(tr) ** 2


def shell_mask(N: int, L: float, lo: float, hi: float) -> np.ndarray:
    n2 = lattice.n2_half(N)
    k = lattice.kf(L) * np.sqrt(n2.astype(np.float64))
    return (n2 > 0) & (k >= lo) & (k < hi)


def shell_sum(Qs: np.ndarray, Qc: np.ndarray, k_b: float, lo: float, hi: float, L: float):
    """S_b = sum over the shell (full grid) of sum_m sum_lambda |e^lambda : X^(m)|^2,
    and N_b, the number of full-grid modes in the shell.  The half layout is
    summed with weight 2 off the kx = 0 and kx = N/2 planes."""
    N = Qs.shape[2]
    mask = shell_mask(N, L, lo, hi)
    w = lattice.half_weights(N)[mask].astype(np.float64)
    nx, ny, nz = lattice.mode_grids_half(N)
    n = np.stack(np.broadcast_arrays(nx, ny, nz), axis=-1)[mask].astype(np.float64)
    khat = n / np.linalg.norm(n, axis=1)[:, None]
    pref = 4.0 / (k_b * k_b)
    s = np.zeros(mask.sum())
    for Qh, sign in ((Qs, -1.0), (Qc, +1.0)):
        X = sym3(sign * pref * Qh[:, mask])
        s += tt_power(X, khat)
    return float(np.sum(w * s)), int(np.sum(w))


def omega_from_sum(S_b: float, N_b: int, k_b: float, L: float) -> float:
    if N_b == 0:
        return 0.0
    V = L ** 3
    return k_b ** 3 * S_b / (48.0 * math.pi ** 2 * V * N_b)


def omega_target(phi_hat, tab_s, tab_c, k_b, lo, hi, L):
    """Omega^(RD)_GW at one target (k_b, shell [lo, hi)) and the shell's mode count."""
    Qs = source_qhat(phi_hat, tab_s, k_b, L)
    Qc = source_qhat(phi_hat, tab_c, k_b, L)
    S, Nb = shell_sum(Qs, Qc, k_b, lo, hi, L)
    return omega_from_sum(S, Nb, k_b, L), Nb


def omega_spectrum(phi_hat, tab_s, tab_c, targets, k_lo, k_hi, L, which=None):
    """Omega at every target (or at the listed target indices), with N_b."""
    idx = range(len(targets)) if which is None else which
    om = np.zeros(len(targets))
    nb = np.zeros(len(targets), dtype=np.int64)
    N = phi_hat.shape[1]
    for b in idx:
        if not shell_mask(N, L, k_lo[b], k_hi[b]).any():
            continue
        om[b], nb[b] = omega_target(phi_hat, tab_s, tab_c, targets[b], k_lo[b], k_hi[b], L)
    return om, nb


def mode_counts(N: int, L: float, k_lo, k_hi) -> np.ndarray:
    w = lattice.half_weights(N)
    return np.array([int(w[shell_mask(N, L, lo, hi)].sum()) for lo, hi in zip(k_lo, k_hi)],
                    dtype=np.int64)
