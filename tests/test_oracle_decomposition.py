"""Pins of the separable decomposition (Sec. V).

P6:
* the grid edges invert the cumulative density of Eq. grid_density, checked
  with an independent adaptive quadrature of rho(u) (not the erf closed form);
* keeping all N_modes eigenpairs rebuilds C_ij / sqrt(L_i L_j) on the strip to
  rounding, the eigenvectors are orthonormal and C q = sigma q;
* the table is ordered by |sigma| and phi_a = q_a / sqrt(L_i);
* E2/E3 diagnostics of the paper's figures: the eigenvalues fall by more than
  an order of magnitude by a = 50, and the 50-term reconstruction is good
  inside the strip away from its edges.
"""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import decomposition, kernels


@pytest.fixture(scope="module")
def tabs():
    return decomposition.tables()


def test_edges_invert_cumulative_density():
    n_modes, u_min, u_max, u_p, s_p, A_p = 200, 1e-3, 15.0, 1.0, 0.5, 10.0
    e = decomposition.grid_edges(n_modes, u_min, u_max, u_p, s_p, A_p)
    rho = lambda u: 1.0 + A_p * math.exp(-(u - u_p) ** 2 / (2 * s_p ** 2))
    total, _ = integrate.quad(rho, u_min, u_max, points=[u_p], epsabs=0, epsrel=1e-13, limit=500)
    for n in (1, 7, 50, 100, 151, 199):
        part, _ = integrate.quad(rho, u_min, e[n], points=[min(u_p, e[n])], epsabs=0, epsrel=1e-13,
                                 limit=500)
        assert abs(part / total * n_modes - n) < 1e-9
    assert e[0] == u_min and e[-1] == u_max
    assert np.all(np.diff(e) > 0)
    # the density bump makes the grid finest near the pivot
    w = np.diff(e)
    c = 0.5 * (e[1:] + e[:-1])
    assert w[np.argmin(np.abs(c - u_p))] < 0.2 * w[-1]


def test_uniform_grid_when_no_bump():
    e = decomposition.grid_edges(10, 1.0, 3.0, 2.0, 0.5, 0.0)
    np.testing.assert_allclose(e, np.linspace(1.0, 3.0, 11), rtol=0, atol=1e-15)


@pytest.mark.parametrize("which", ["s", "c"])
def test_full_eigen_reconstruction(tabs, which):
    t = tabs[0] if which == "s" else tabs[1]
    C = decomposition.kernel_matrix(t.edges, which)
    Q, w = t.q_all, t.sigma_all
    np.testing.assert_allclose(Q.T @ Q, np.eye(len(w)), atol=1e-12)
    assert np.linalg.norm(C @ Q - Q * w) <= 1e-12 * np.linalg.norm(C)
    L = np.diff(t.edges)
    K = C / np.sqrt(np.outer(L, L))
    R = t.reconstruct(len(w))
    assert np.max(np.abs(R - K)) <= 1e-11 * np.max(np.abs(K))
    # ordering and the phi definition
    assert np.all(np.diff(np.abs(w)) <= 1e-12)
    np.testing.assert_allclose(t.phi, Q[:, :50] / np.sqrt(L)[:, None], rtol=0, atol=0)


@pytest.mark.parametrize("which", ["s", "c"])
def test_strip_and_kernel_values(tabs, which):
    t = tabs[0] if which == "s" else tabs[1]
    C = decomposition.kernel_matrix(t.edges, which)
    c = 0.5 * (t.edges[1:] + t.edges[:-1])
    L = np.diff(t.edges)
    f = kernels.I_s if which == "s" else kernels.I_c
    i, j = 60, 75
    if abs(c[i] - c[j]) <= 1 <= c[i] + c[j]:
        assert C[i, j] == pytest.approx(math.sqrt(L[i] * L[j]) * float(f(c[i], c[j])), rel=1e-14)
    assert C[0, 199] == 0.0          # |u - v| > 1: outside the triangle strip
    assert C[0, 1] == 0.0            # u + v < 1: outside the triangle strip
    assert np.all(np.isfinite(C))
    np.testing.assert_array_equal(C, C.T)


@pytest.mark.parametrize("which", ["s", "c"])
def test_eigenvalue_falloff_and_reconstruction(tabs, which):
    """Fig. eigenvalues / Fig. reconstruction: |sigma_50|/|sigma_1| well below 1,
    and the 50-term kernel close to the full one away from the strip edges."""
    t = tabs[0] if which == "s" else tabs[1]
    assert abs(t.sigma[49] / t.sigma[0]) < 0.1
    L = np.diff(t.edges)
    K = decomposition.kernel_matrix(t.edges, which) / np.sqrt(np.outer(L, L))
    R = t.reconstruct(50)
    c = 0.5 * (t.edges[1:] + t.edges[:-1])
    U, V = np.meshgrid(c, c, indexing="ij")
    inner = (np.abs(U - V) <= 0.8) & (U + V >= 1.3) & (U + V <= 6)
    rel = np.abs(R - K)[inner] / np.max(np.abs(K[inner]))
    assert np.median(rel) < 0.05
