"""Direct O(N^6) mode sums of the envelope integrals (Eq. naive_A, naive_B).

With  int d^3q/(2 pi)^3 -> (1/V) sum_n  and  (2 pi)^3 delta(q) -> V delta_n,
the convolution evaluated by the FFT engine is, for each output mode n,

    Q_hat_ij(n) = -(1/V) sum_{n1} qt_i(n1) qt_j(n2) K(u(n1), u(n2)) Phi_hat(n1) Phi_hat(n2)

with n2 = n - n1 and the -1 from (i q)(i q).  ``truncated`` uses the kept
separable kernel K = sum_{a<N_alpha} sigma_a phi_a phi_a and the periodic
wrap n2 = (n - n1) mod N (the sum the FFTs compute, term for term);
``exact`` uses the closed-form I_s / I_c of Eq. kernels and no wrap (terms
with n2 off the lattice dropped), restricted like the decomposition to the
triangle strip |u - v| <= 1 <= u + v; u and v are |q|/k with k the target
k_b, as in the method, or the output mode's own |k| when k_b is None.
"""
from __future__ import annotations

import numpy as np

from . import kernels, lattice


def full_from_half(Xh: np.ndarray) -> np.ndarray:
    """Rebuild the full spectrum from the half layout using X(-n) = X(n)*."""
    N = Xh.shape[1]
    H = N // 2 + 1
    full = np.empty((N, N, N), dtype=np.complex128)
    full[:H] = Xh
    for kx in range(H, N):
        src = N - kx
        full[kx] = np.conj(Xh[src][(-np.arange(N)) % N][:, (-np.arange(N)) % N])
    return full


def _qt_full(N, L):
    n = lattice.signed_full(N).astype(np.float64)
    q = lattice.kf(L) * n
    q = np.where(lattice.signed_full(N) == -(N // 2), 0.0, q)
    return q


def truncated_qhat(phi_hat_half: np.ndarray, table, k_b: float, L: float, out_modes):
    """Q_hat_ij at the given (kx, ky, kz) full-grid index triples."""
    N = phi_hat_half.shape[1]
    V = L ** 3
    F = full_from_half(phi_hat_half).reshape(-1)
    n = lattice.signed_full(N)
    ix, iy, iz = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
    ix, iy, iz = ix.ravel(), iy.ravel(), iz.ravel()
    n2 = (n[ix] ** 2 + n[iy] ** 2 + n[iz] ** 2).astype(np.float64)
    u = lattice.kf(L) * np.sqrt(n2) / k_b
    idx = table.interval_index(u)
    # kept kernel on the intervals, with a zero row/column for "outside"
    Lw = table.edges[1:] - table.edges[:-1]
    Kfull = np.zeros((len(Lw) + 1, len(Lw) + 1))
    Kfull[:-1, :-1] = (table.phi * table.sigma) @ table.phi.T
    idx = np.where(idx >= 0, idx, len(Lw))
    q = _qt_full(N, L)
    qs = (q[ix], q[iy], q[iz])
    out = np.zeros((6, len(out_modes)), dtype=np.complex128)
    pairs = ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))
    for o, (ox, oy, oz) in enumerate(out_modes):
        jx = (ox - ix) % N
        jy = (oy - iy) % N
        jz = (oz - iz) % N
        j = (jx * N + jy) * N + jz
        base = Kfull[idx, idx[j]] * F * F[j]
        for c, (a, b) in enumerate(pairs):
            out[c, o] = -np.sum(qs[a] * qs[b][j] * base) / V
    return out


def exact_qhat(phi_hat_half: np.ndarray, which: str, L: float, out_modes, k_b=None):
    """Q_hat_ij with the closed-form kernel, no wrap."""
    N = phi_hat_half.shape[1]
    V = L ** 3
    F = full_from_half(phi_hat_half).reshape(-1)
    n = lattice.signed_full(N)
    ix, iy, iz = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
    ix, iy, iz = ix.ravel(), iy.ravel(), iz.ravel()
    k = lattice.kf(L)
    q1 = np.stack([k * n[ix], k * n[iy], k * n[iz]], axis=1).astype(np.float64)
    f = kernels.I_s if which == "s" else kernels.I_c
    out = np.zeros((6, len(out_modes)), dtype=np.complex128)
    pairs = ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))
    half = N // 2
    for o, (ox, oy, oz) in enumerate(out_modes):
        no = np.array([n[ox], n[oy], n[oz]], dtype=np.int64)
        kout = k * np.sqrt(float(no @ no)) if k_b is None else k_b
        m2 = no[None, :] - np.stack([n[ix], n[iy], n[iz]], axis=1)
        inside = np.all((m2 >= -half) & (m2 < half), axis=1)
        m2i = np.where(inside[:, None], m2 % N, 0)
        j = (m2i[:, 0] * N + m2i[:, 1]) * N + m2i[:, 2]
        q2 = k * m2.astype(np.float64)
        u = np.linalg.norm(q1, axis=1) / kout
        v = np.linalg.norm(q2, axis=1) / kout
        ok = inside & (u > 0) & (v > 0) & (np.abs(u - v) <= 1.0) & (u + v >= 1.0)
        with np.errstate(all="ignore"):
            Kv = np.where(ok, f(np.where(ok, u, 1.0), np.where(ok, v, 1.0)), 0.0)
        base = Kv * F * np.where(ok, F[j], 0.0)
        for c, (a, b) in enumerate(pairs):
            out[c, o] = -np.sum(q1[:, a] * q2[:, b] * base) / V
    return out
