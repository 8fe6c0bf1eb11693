"""Separable decomposition of the kernels (Sec. V).

Steps, in the order of Sec. V:
1. Non-uniform u-grid from the density rho(u) = 1 + A_p exp(-(u-u_p)^2/(2 sigma_p^2))
   (Eq. grid_density): the normalised cumulative n(u) is inverted at
   n = 0..N_modes, giving N_modes intervals [e_i, e_{i+1}) with centres
   c_i (midpoints) and widths L_i.
2. Indicator basis f_i = 1_i / sqrt(L_i) (Eq. basis) and the kernel matrix
   C_ij ~ sqrt(L_i L_j) I(c_i, c_j) (Eq. C_matrix_discrete), restricted to the
   strip where u, v and the unit vector k-hat can close a triangle:
   |c_i - c_j| <= 1 <= c_i + c_j (the printed "|u +- v| < 1" cannot be meant
   literally, since then no pair with u + v > 1 would survive).
3. Symmetric eigendecomposition C = sum_a sigma_a q_a q_a^T (Eq. diagonalization),
   ordered by |sigma| descending; the N_alpha largest are kept, with their signs.
4. phi_a(u) = sum_i q_a,i f_i(u), i.e. q_a,i / sqrt(L_i) on interval i and zero
   outside [u_min, u_max).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
from scipy.special import erf

from . import kernels


def grid_cumulative(u, u_min, u_p, sigma_p, A_p):
    """int_{u_min}^{u} rho(u') du' for rho = 1 + A_p exp(-(u-u_p)^2/(2 sigma_p^2))."""
    s2 = math.sqrt(2.0) * sigma_p
    return (u - u_min) + A_p * sigma_p * math.sqrt(math.pi / 2.0) * (
        erf((u - u_p) / s2) - erf((u_min - u_p) / s2))


def grid_edges(n_modes, u_min, u_max, u_p, sigma_p, A_p) -> np.ndarray:
    """Edges e_n = n^{-1}(n), n = 0..N_modes, of Eq. grid_density.  Each edge is
    the smallest double at which the cumulative reaches its share, found by
    bisection down to adjacent doubles."""
    total = grid_cumulative(u_max, u_min, u_p, sigma_p, A_p)
    e = np.empty(n_modes + 1, dtype=np.float64)
    e[0] = u_min
    e[n_modes] = u_max
    for n in range(1, n_modes):
        target = total * n / n_modes
        lo, hi = u_min, u_max
        while True:
            mid = 0.5 * (lo + hi)
            if mid <= lo or mid >= hi:
                break
            if grid_cumulative(mid, u_min, u_p, sigma_p, A_p) < target:
                lo = mid
            else:
                hi = mid
        e[n] = hi
    return e


def kernel_matrix(edges: np.ndarray, which: str, kernel=None) -> np.ndarray:
    """C_ij = sqrt(L_i L_j) I(c_i, c_j) inside the triangle strip, else 0.
    I is I_s or I_c of Eq. kernels, or the callable kernel(u, v) if given
    (another kernel on the same strip, e.g. from another equation of
    state)."""
    c = 0.5 * (edges[:-1] + edges[1:])
    L = edges[1:] - edges[:-1]
    U, Vv = np.meshgrid(c, c, indexing="ij")
    strip = (np.abs(U - Vv) <= 1.0) & (U + Vv >= 1.0)
    f = kernel if kernel is not None else (kernels.I_s if which == "s" else kernels.I_c)
    with np.errstate(all="ignore"):
        K = np.where(strip, f(U, Vv), 0.0)
    return np.sqrt(np.outer(L, L)) * K


@dataclass
class KernelTable:
    which: str
    edges: np.ndarray      # N_modes + 1
    sigma: np.ndarray      # N_alpha, ordered by |sigma| descending
    phi: np.ndarray        # N_modes x N_alpha, phi_a on interval i
    sigma_all: np.ndarray  # all N_modes eigenvalues, same order
    q_all: np.ndarray      # all eigenvectors (columns), same order

    def reconstruct(self, n_keep=None) -> np.ndarray:
        """sum_{a<n_keep} sigma_a phi_a(c_i) phi_a(c_j) on the interval centres."""
        n = len(self.sigma) if n_keep is None else n_keep
        L = self.edges[1:] - self.edges[:-1]
        Q = self.q_all[:, :n] / np.sqrt(L)[:, None]
        return (Q * self.sigma_all[:n]) @ Q.T

    def interval_index(self, u: np.ndarray) -> np.ndarray:
        """Index i with e_i <= u < e_{i+1}; -1 outside [u_min, u_max)."""
        idx = np.searchsorted(self.edges, u, side="right") - 1
        ok = (u >= self.edges[0]) & (u < self.edges[-1])
        return np.where(ok, idx, -1)


def decompose(which: str, n_modes=200, n_alpha=50, u_min=1e-3, u_max=15.0,
              u_p=1.0, sigma_p=0.5, A_p=10.0, kernel=None) -> KernelTable:
    edges = grid_edges(n_modes, u_min, u_max, u_p, sigma_p, A_p)
    C = kernel_matrix(edges, which, kernel)
    w, Q = np.linalg.eigh(C)
    order = np.argsort(-np.abs(w), kind="stable")
    w = w[order]
    Q = Q[:, order]
    L = edges[1:] - edges[:-1]
    phi = Q[:, :n_alpha] / np.sqrt(L)[:, None]
    return KernelTable(which=which, edges=edges, sigma=w[:n_alpha].copy(), phi=phi,
                       sigma_all=w, q_all=Q)


def tables(decomp=None):
    """Both kernel tables (sine, cosine) for a Decomposition of meta-parameters."""
    kw = {} if decomp is None else dict(
        n_modes=decomp.n_modes, n_alpha=decomp.n_alpha, u_min=decomp.u_min,
        u_max=decomp.u_max, u_p=decomp.u_p, sigma_p=decomp.sigma_p, A_p=decomp.A_p)
    return decompose("s", **kw), decompose("c", **kw)
