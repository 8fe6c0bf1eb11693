"""Time-integral kernels of the asymptotic envelopes (Sec. IV).

The radiation-era potential transfer function is T(x) = 3 j_1(y)/y with
y = x/sqrt(3) (Sec. II, w = 1/3).  The envelope integrals define

    I_s(u, v) = int_0^inf dt t sin(t) f(t, u, v)
    I_c(u, v) = int_0^inf dt t cos(t) f(t, u, v)
    f(t, u, v) = T(ut) T(vt) + 1/2 (T + t dT/dt)(ut) (T + t dT/dt)(vt)

(the printed f repeats T(q_1); the second factor is T(q_2), as in the
dimensionless form of Sec. IV).  Their closed forms (Eq. kernels) are what the
method decomposes; the quadrature forms here exist only to pin the closed
forms in the tests.
"""
from __future__ import annotations

import math

import numpy as np

SQRT3 = math.sqrt(3.0)


def I_s(u, v):
    """Eq. kernels, sine kernel: 27 pi (u^2+v^2-3)^2 / (32 u^3 v^3) Theta(u+v-sqrt3)."""
    u = np.asarray(u, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    a = u * u + v * v - 3.0
    val = 27.0 * math.pi * a * a / (32.0 * u ** 3 * v ** 3)
    return np.where(u + v > SQRT3, val, 0.0)


def I_c(u, v):
    """Eq. kernels, cosine kernel:
    27 (u^2+v^2-3) / (32 u^3 v^3) [ -4uv + (u^2+v^2-3) ln|(3-(u+v)^2)/(3-(u-v)^2)| ]."""
    u = np.asarray(u, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    a = u * u + v * v - 3.0
    with np.errstate(divide="ignore"):
        lg = np.log(np.abs((3.0 - (u + v) ** 2) / (3.0 - (u - v) ** 2)))
    return 27.0 * a / (32.0 * u ** 3 * v ** 3) * (-4.0 * u * v + a * lg)


def transfer(x):
    """T(x) = 3 j_1(y)/y, y = x/sqrt(3): the w = 1/3 potential transfer function."""
    y = np.asarray(x, dtype=np.float64) / SQRT3
    out = np.empty_like(y)
    small = np.abs(y) < 1e-3
    ys = y[small]
    out[small] = 1.0 - ys * ys / 10.0 + ys ** 4 / 280.0
    yl = y[~small]
    out[~small] = 3.0 * (np.sin(yl) - yl * np.cos(yl)) / yl ** 3
    return out


def transfer_plus(x):
    """T + x dT/dx evaluated at x (the (T + H^{-1} T') factor with H = 1/eta)."""
    y = np.asarray(x, dtype=np.float64) / SQRT3
    out = np.empty_like(y)
    small = np.abs(y) < 1e-3
    ys = y[small]
    # d/dy [y T] = T + y T'; series of 3 j1(y)/y = 1 - y^2/10 + y^4/280
    out[small] = 1.0 - 3.0 * ys * ys / 10.0 + 5.0 * ys ** 4 / 280.0
    yl = y[~small]
    s, c = np.sin(yl), np.cos(yl)
    T = 3.0 * (s - yl * c) / yl ** 3
    dT = 3.0 * (yl * yl * s + 3.0 * yl * c - 3.0 * s) / yl ** 4
    out[~small] = T + yl * dT
    return out


def source_kernel(t, u, v):
    """f(t, u, v) = T(ut)T(vt) + 1/2 (T + t dT/dt)(ut) (T + t dT/dt)(vt)."""
    t = np.asarray(t, dtype=np.float64)
    return transfer(u * t) * transfer(v * t) + 0.5 * transfer_plus(u * t) * transfer_plus(v * t)


def time_integral(u: float, v: float, which: str, eps_list=(0.01, 0.005, 0.0025),
                  t_max_factor: float = 60.0, n_per_unit: int = 80) -> float:
    """int_0^inf dt t {sin, cos}(t) f(t,u,v), with an exp(-eps t) damping and
    Richardson extrapolation eps -> 0 over a quadratic fit.  Used only to pin
    the closed forms of Eq. kernels."""
    trig = np.sin if which == "s" else np.cos
    vals = []
    for eps in eps_list:
        tmax = t_max_factor / eps
        n = int(tmax * n_per_unit) | 1
        t = np.linspace(0.0, tmax, n)
        g = t * trig(t) * source_kernel(t, u, v) * np.exp(-eps * t)
        h = t[1] - t[0]
        # composite Simpson
        vals.append(h / 3.0 * (g[0] + g[-1] + 4.0 * g[1:-1:2].sum() + 2.0 * g[2:-1:2].sum()))
    e = np.asarray(eps_list)
    A = np.vstack([np.ones_like(e), e, e * e]).T
    coef = np.linalg.solve(A, np.asarray(vals))
    return float(coef[0])
