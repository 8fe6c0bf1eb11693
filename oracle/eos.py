"""Envelope kernels for a background of constant equation of state w (Sec. II,
Sec. IV), the kernel-table variant the paper names as the extension of its
method to other thermal histories.  TEST INFRASTRUCTURE (see oracle/__init__).

Sec. II states the equations for any expansion history and then fixes
w = 1/3.  For a constant w with adiabatic pressure (c_s^2 = w) they solve as
follows (b = (1 - 3w)/(1 + 3w), a ~ eta^(1+b), conformal Hubble
H = (1 + b)/eta):

* Eq. scalar with nabla^2 -> -k^2: the mass term 2H' + (1 + 3w) H^2 vanishes,
  leaving T'' + (p/eta) T' + w k^2 T = 0 with p = 6(1 + w)/(1 + 3w) and
  T(0) = 1, T'(0) = 0.  So T(eta, k) = Tn(sqrt(w) k eta) with
  Tn(x) = Gamma(nu + 1) (2/x)^nu J_nu(x), nu = (p - 1)/2 = (5 + 3w)/(2(1 + 3w)).
* The homogeneous wave equation y'' + 2H y' + k^2 y = 0, in t = k eta:
  y2(t) = sqrt(pi/2) t^-mu J_mu(t), y1(t) = -sqrt(pi/2) t^-mu Y_mu(t),
  mu = b + 1/2, with Wronskian W = y1 y2' - y1' y2 = k t^(-2(1+b)), which
  falls as a^-2 (Abel's identity).
* Eq. envelopes, A' = -y2 S / W and B' = y1 S / W, integrated to eta -> inf
  with the source of Sec. I in the variables u = q1/k, v = q2/k of Sec. IV:
  A = 4 k^3 e^ij int int ... u_i v_j Phi Phi I_s^w(u, v) and B likewise with
  -I_c^w, where
      I_s^w(u, v) = r^2 int_0^inf dt t^(2(1+b)) y2(t) f(t, u, v),
      I_c^w(u, v) = r^2 int_0^inf dt t^(2(1+b)) y1(t) f(t, u, v),
      f(t, u, v) = T(ut) T(vt) + 2/(3(1 + w)) D(ut) D(vt),
      D = T + H^-1 dT/deta = Tn(x) + x Tn'(x) / (1 + b),  x = sqrt(w) u t.
  The initial potential is Phi_i = 3(1 + w)/(5 + 3w) zeta (Sec. II); the
  lattice path carries Phi = 2 zeta / 3, so the kernels take the factor
  r = [3(1 + w)/(5 + 3w)] / (2/3).
* At w = 1/3: b = 0, nu = 3/2, mu = 1/2, r = 1, Tn(x) = 3 j1(x)/x,
  t^2 y2 = t sin t, t^2 y1 = t cos t, and I^w are the I_s, I_c of Sec. IV,
  whose closed forms are Eq. kernels.
The late-time relation between the envelopes and Omega for w != 1/3 (the
w = 1/3 form is Sec. III) is not part of this module.

Evaluation of int_0^inf (all products of Bessel functions, decaying like a
power and oscillating with frequencies 1 +- sqrt(w) u +- sqrt(w) v, near zero
close to the resonance sqrt(w)(u + v) = 1):
* [0, T1]: composite Gauss-Legendre panels (the first panel graded towards
  t = 0), with T1 such that sqrt(w) u T1 >= 12 for every u on the grid;
* [T1, inf): each real Bessel factor is the real part of a Hankel function
  H1 (J = Re H1, Y = Im H1 on the real line), so the product of the three
  factors is 1/4 Re of four analytic products, each carrying one frequency
  Omega; each is integrated along the ray t = T1 + i sign(Omega) s, where it
  decays like exp(-|Omega| s), with a double-exponential (exp-sinh) rule in
  s.  The Hankel functions are SciPy's (AMOS), evaluated at complex points.
"""
from __future__ import annotations

import math

import numpy as np
from numpy.polynomial.legendre import leggauss
from scipy import special

from . import decomposition


def params(w: float):
    """(b, nu, mu, c_src, r) of the constant-w background (module docstring)."""
    if not (0.0 < w < 1.0):
        raise ValueError("w must lie in (0, 1)")
    b = (1.0 - 3.0 * w) / (1.0 + 3.0 * w)
    nu = (5.0 + 3.0 * w) / (2.0 * (1.0 + 3.0 * w))
    mu = b + 0.5
    c_src = 2.0 / (3.0 * (1.0 + w))
    r = (3.0 * (1.0 + w) / (5.0 + 3.0 * w)) / (2.0 / 3.0)
    return b, nu, mu, c_src, r


def transfer(x, w):
    """Tn(x) = Gamma(nu+1) (2/x)^nu J_nu(x): the potential's transfer function
    T(eta, k) = Tn(sqrt(w) k eta), Tn(0) = 1."""
    _, nu, _, _, _ = params(w)
    x = np.asarray(x, dtype=np.float64)
    g = math.gamma(nu + 1.0) * 2.0 ** nu
    with np.errstate(divide="ignore", invalid="ignore"):
        out = g * x ** (-nu) * special.jv(nu, x)
    return np.where(x == 0.0, 1.0, out)


def transfer_D(x, w):
    """D(x) = Tn(x) + x Tn'(x)/(1 + b) = Gamma(nu+1) 2^nu x^-nu [J_nu(x) - x J_(nu+1)(x)/(1 + b)]
    (using d/dx [x^-nu J_nu] = -x^-nu J_(nu+1)): the factor T + H^-1 dT/deta."""
    b, nu, _, _, _ = params(w)
    x = np.asarray(x, dtype=np.float64)
    g = math.gamma(nu + 1.0) * 2.0 ** nu
    with np.errstate(divide="ignore", invalid="ignore"):
        out = g * x ** (-nu) * (special.jv(nu, x) - x * special.jv(nu + 1.0, x) / (1.0 + b))
    return np.where(x == 0.0, 1.0, out)


def y_solutions(t, w):
    """(y1, y2) at t = k eta: the two solutions of the homogeneous wave equation."""
    _, _, mu, _, _ = params(w)
    t = np.asarray(t, dtype=np.float64)
    c = math.sqrt(math.pi / 2.0) * t ** (-mu)
    return -c * special.yv(mu, t), c * special.jv(mu, t)


# -------------------------------------------------------------- quadrature
def _gl_nodes(T1: float, h: float = 0.5, n: int = 24, grade: int = 24):
    """Gauss-Legendre nodes and weights on [0, T1]: panels of width h, the
    first one split geometrically towards t = 0 (the integrand has a
    non-analytic power t^(1 + 2 mu) there)."""
    xg, wg = leggauss(n)
    edges = [0.0] + [h * 2.0 ** (-k) for k in range(grade, 0, -1)] + list(np.arange(h, T1 + 0.5 * h, h))
    edges = np.asarray(edges)
    a, c = edges[:-1], edges[1:]
    t = (0.5 * (c - a))[:, None] * xg[None, :] + (0.5 * (c + a))[:, None]
    wt = (0.5 * (c - a))[:, None] * wg[None, :]
    return t.ravel(), wt.ravel()


def _expsinh_nodes(h: float = 1.0 / 24.0, xmax: float = 4.5):
    """exp-sinh rule for int_0^inf g(s) ds: s = exp(pi/2 sinh x)."""
    x = np.arange(-xmax, xmax + 0.5 * h, h)
    s = np.exp(0.5 * math.pi * np.sinh(x))
    ws = h * 0.5 * math.pi * np.cosh(x) * s
    return s, ws


def _amplitudes(xc, w):
    """Non-oscillating parts of the Hankel forms at complex x (Z = e^{ix} P):
    P_T(x) = Gamma(nu+1) 2^nu x^-nu h1e(nu, x) and
    P_D(x) = Gamma(nu+1) 2^nu x^-nu [h1e(nu, x) - x h1e(nu+1, x)/(1 + b)],
    with h1e(nu, x) = H1_nu(x) exp(-ix)."""
    b, nu, _, _, _ = params(w)
    g = math.gamma(nu + 1.0) * 2.0 ** nu
    xp = xc ** (-nu)
    h0 = special.hankel1e(nu, xc)
    h1 = special.hankel1e(nu + 1.0, xc)
    return g * xp * h0, g * xp * (h0 - xc * h1 / (1.0 + b))


def kernel_matrices(c, w, T1=None, panel=0.5, gl_n=24, es_h=1.0 / 24.0):
    """(I_s^w, I_c^w) at every pair of the points c (1-D array, all > 0), as
    two len(c) x len(c) matrices (module docstring for the definitions and
    the method)."""
    b, nu, mu, c_src, r = params(w)
    c = np.asarray(c, dtype=np.float64)
    alpha = math.sqrt(w) * c
    if T1 is None:
        T1 = panel * math.ceil(12.0 / alpha.min() / panel)
    n = len(c)
    Is = np.zeros((n, n))
    Ic = np.zeros((n, n))
    # [0, T1]: f = T T + c_src D D is a sum of two separable products, so the
    # quadrature is a pair of matrix products
    t, wt = _gl_nodes(T1, panel, gl_n)
    for s0 in range(0, len(t), 8192):
        tb, wb = t[s0:s0 + 8192], wt[s0:s0 + 8192]
        X = alpha[:, None] * tb[None, :]
        Tv = transfer(X, w)
        Dv = transfer_D(X, w)
        y1, y2 = y_solutions(tb, w)
        pw = tb ** (2.0 * (1.0 + b))
        for M, yv in ((Is, y2), (Ic, y1)):
            g = wb * pw * yv
            M += (Tv * g) @ Tv.T + c_src * ((Dv * g) @ Dv.T)
    # [T1, inf): rays t = T1 +- i s; beyond |Omega| s = 745 every term is
    # below the smallest double, so the rule stops there
    om_min = min(np.abs(1.0 + sa * alpha[:, None] + sb * alpha[None, :]).min()
                 for sa in (+1, -1) for sb in (+1, -1))
    s, ws = _expsinh_nodes(es_h)
    keep = s * om_min <= 745.0
    s, ws = s[keep], ws[keep]
    z_up = T1 + 1j * s
    z_dn = T1 - 1j * s
    PT_up, PD_up = _amplitudes(alpha[:, None] * z_up[None, :], w)
    PT_dn, PD_dn = _amplitudes(alpha[:, None] * z_dn[None, :], w)
    ymu = math.sqrt(math.pi / 2.0)
    Py_up = ymu * z_up ** (-mu) * special.hankel1e(mu, z_up) * z_up ** (2.0 * (1.0 + b))
    Py_dn = ymu * z_dn ** (-mu) * special.hankel1e(mu, z_dn) * z_dn ** (2.0 * (1.0 + b))
    tail_s = np.zeros((n, n), dtype=np.complex128)
    tail_c = np.zeros((n, n), dtype=np.complex128)
    for sa in (+1, -1):
        for sb in (+1, -1):
            Om = 1.0 + sa * alpha[:, None] + sb * alpha[None, :]
            up = Om > 0.0
            for P_up, P_dn, coef in ((PT_up, PT_dn, 1.0), (PD_up, PD_dn, c_src)):
                # factor a at z: P(alpha z) for sign +, conj(P(alpha conj z)) for sign -
                A_up = P_up if sa > 0 else np.conj(P_dn)
                A_dn = P_dn if sa > 0 else np.conj(P_up)
                B_up = P_up if sb > 0 else np.conj(P_dn)
                B_dn = P_dn if sb > 0 else np.conj(P_up)
                acc_up = np.zeros((n, n), dtype=np.complex128)
                acc_dn = np.zeros((n, n), dtype=np.complex128)
                for k in range(len(s)):
                    x = np.abs(Om) * s[k]
                    E = np.where(x < 745.0, np.exp(-np.minimum(x, 745.0)), 0.0)
                    acc_up += (ws[k] * Py_up[k]) * E * np.outer(A_up[:, k], B_up[:, k])
                    acc_dn += (ws[k] * Py_dn[k]) * E * np.outer(A_dn[:, k], B_dn[:, k])
                ph = np.exp(1j * Om * T1)
                contrib = coef * ph * np.where(up, 1j * acc_up, -1j * acc_dn)
                tail_s += contrib
                tail_c += 1j * contrib            # y1 = Re(i Z_y) where y2 = Re(Z_y)
    Is += 0.25 * tail_s.real
    Ic += 0.25 * tail_c.real
    return r * r * Is, r * r * Ic


def strip_kernels(w, **kw):
    """(kernel_s, kernel_c): callables kernel(U, V) for
    decomposition.decompose(..., kernel=...) that return I_s^w or I_c^w on
    the meshgrid of the interval centres; both share one evaluation of the
    time integrals."""
    cache = {}

    def make(which):
        def kernel(U, V):
            c = U[:, 0]
            assert np.array_equal(V[0, :], c), "called on the meshgrid of the interval centres"
            key = c.tobytes()
            if key not in cache:
                cache[key] = kernel_matrices(c, w, **kw)
            return cache[key][0 if which == "s" else 1]
        return kernel

    return make("s"), make("c")


def tables_w(w, n_modes=200, n_alpha=50, u_min=1e-3, u_max=15.0, u_p=1.0, sigma_p=0.5, A_p=10.0):
    """Both separable tables (Sec. V) of the constant-w kernels on the grid
    of these meta-parameters."""
    ks, kc = strip_kernels(w)
    kw = dict(n_modes=n_modes, n_alpha=n_alpha, u_min=u_min, u_max=u_max, u_p=u_p, sigma_p=sigma_p, A_p=A_p)
    return decomposition.decompose("s", kernel=ks, **kw), decomposition.decompose("c", kernel=kc, **kw)


def time_integral_damped(u: float, v: float, w: float, which: str, eps_list=(0.02, 0.01, 0.005),
                         t_max_factor: float = 50.0, n_per_unit: int = 60) -> float:
    """The same kernel by a different route, for pinning: exp(-eps t) damping
    of the plain real-line integral, composite Simpson, and a quadratic
    extrapolation eps -> 0.  Accurate to ~1e-4 away from the resonance."""
    b, nu, mu, c_src, r = params(w)
    a, bb = math.sqrt(w) * u, math.sqrt(w) * v
    vals = []
    for eps in eps_list:
        tmax = t_max_factor / eps
        nn = int(tmax * n_per_unit) | 1
        t = np.linspace(1e-12, tmax, nn)
        y1, y2 = y_solutions(t, w)
        f = transfer(a * t, w) * transfer(bb * t, w) + c_src * transfer_D(a * t, w) * transfer_D(bb * t, w)
        g = t ** (2.0 * (1.0 + b)) * (y2 if which == "s" else y1) * f * np.exp(-eps * t)
        h = t[1] - t[0]
        vals.append(h / 3.0 * (g[0] + g[-1] + 4.0 * g[1:-1:2].sum() + 2.0 * g[2:-1:2].sum()))
    e = np.asarray(eps_list)
    A = np.vstack([np.ones_like(e), e, e * e]).T
    return float(r * r * np.linalg.solve(A, np.asarray(vals))[0])
