// Envelope kernels for a background of constant equation of state w (Sec. II
// equations, Sec. IV time integrals), evaluated on the host for the
// separable tables of Sec. V.
//
// With b = (1 - 3w)/(1 + 3w) (a ~ eta^(1+b), conformal Hubble (1 + b)/eta)
// and adiabatic pressure (c_s^2 = w):
//   potential transfer    T(eta, k) = Tn(sqrt(w) k eta),
//                         Tn(x) = Gamma(nu + 1) (2/x)^nu J_nu(x), nu = (5 + 3w)/(2(1 + 3w))
//                         (Eq. scalar loses its mass term for constant w);
//   tensor Green's pair   y2(t) = sqrt(pi/2) t^-mu J_mu(t), y1(t) = -sqrt(pi/2) t^-mu Y_mu(t),
//                         mu = b + 1/2, t = k eta, Wronskian k t^(-2(1+b)) (Abel);
//   kernels               I_s^w = r^2 int_0^inf dt t^(2(1+b)) y2 f,  I_c^w = the same with y1,
//                         f = T(ut) T(vt) + 2/(3(1+w)) D(ut) D(vt),
//                         D(x) = Tn(x) + x Tn'(x)/(1 + b),
//                         r = [3(1+w)/(5+3w)] / (2/3) (Phi_i of Sec. II over the 2/3 the
//                         lattice path applies to zeta).
// At w = 1/3 these are the I_s, I_c of Sec. IV (Eq. kernels).
//
// Numerics (double precision throughout):
//   * Tn, D, y2 below x = kSwitch from their power series, above it from the
//     asymptotic (Hankel) expansion; y1 below kSwitch by integrating its ODE
//     y'' + 2(1 + b)/t y' + y = 0 in s = ln t from kSwitch down to the
//     smallest node (the direction in which y1 dominates);
//   * [0, T1]: composite Gauss-Legendre, T1 such that sqrt(w) u T1 >= kTail
//     for the smallest u, so every factor is in its asymptotic range beyond;
//   * [T1, inf): each factor is the real part of its Hankel form, the product
//     of three is 1/4 Re of four analytic terms with frequencies
//     1 +- sqrt(w) u +- sqrt(w) v; each is integrated along t = T1 + i sign s
//     with a double-exponential rule, on which it decays like exp(-|freq| s).
#include <algorithm>
#include <cmath>
#include <complex>
#include <stdexcept>
#include <vector>

#include "sigw_eos.hpp"

namespace sigw {
namespace {

using cd = std::complex<double>;
constexpr double kPi = 3.14159265358979323846;
constexpr double kSwitch = 14.0;   // series below, asymptotic expansion above
constexpr double kTail = 14.0;     // sqrt(w) u_min T1 >= kTail

struct Bg {
    double w, b, nu, mu, csrc, r, g_nu, g_nu1;
};

Bg background(double w) {
    Bg g;
    g.w = w;
    g.b = (1.0 - 3.0 * w) / (1.0 + 3.0 * w);
    g.nu = (5.0 + 3.0 * w) / (2.0 * (1.0 + 3.0 * w));
    g.mu = g.b + 0.5;
    g.csrc = 2.0 / (3.0 * (1.0 + w));
    g.r = (3.0 * (1.0 + w) / (5.0 + 3.0 * w)) / (2.0 / 3.0);
    g.g_nu = std::tgamma(g.nu + 1.0) * std::pow(2.0, g.nu);
    g.g_nu1 = std::tgamma(g.nu + 2.0) * std::pow(2.0, g.nu + 1.0);
    return g;
}

// sum_k (-x^2/4)^k Gamma(a+1) / (k! Gamma(a+k+1)) = Gamma(a+1) (2/x)^a J_a(x)
double bessel_norm_series(double a, double x) {
    const double q = -0.25 * x * x;
    double term = 1.0, sum = 1.0;
    for (int k = 1; k < 400; ++k) {
        term *= q / (double(k) * (a + double(k)));
        sum += term;
        if (std::fabs(term) < 1e-18 * std::fabs(sum) && k > 4) break;
    }
    return sum;
}

// Asymptotic (Hankel) expansion: H1_a(z) = sqrt(2/(pi z)) exp(i(z - a pi/2 - pi/4)) S_a(z),
// S_a(z) = sum_k i^k c_k(a) z^-k, c_k = prod_{j<=k} (4a^2 - (2j-1)^2) / (k! 8^k),
// summed until the terms stop decreasing or fall below 1e-17.  Returns
// P_a(z) = sqrt(2/(pi z)) exp(-i(a pi/2 + pi/4)) S_a(z), so H1_a(z) = e^{iz} P_a(z).
cd hankel_amp(double a, cd z) {
    const double m = 4.0 * a * a;
    cd sum = 1.0, term = 1.0;
    const cd iz = cd(0.0, 1.0) / z;
    double last = 1.0;
    for (int k = 1; k < 200; ++k) {
        const double c = (m - double(2 * k - 1) * (2 * k - 1)) / (8.0 * k);
        const cd next = term * c * iz;
        const double mag = std::abs(next);
        if (mag > last) break;            // asymptotic series: stop at the smallest term
        term = next;
        sum += term;
        last = mag;
        if (mag < 1e-17 * std::abs(sum)) break;
    }
    return std::sqrt(2.0 / (kPi * z)) * std::exp(cd(0.0, -(a * kPi / 2.0 + kPi / 4.0))) * sum;
}

// Tn(x), D(x) at real x >= 0
void transfer_pair(const Bg& g, double x, double* T, double* D) {
    if (x < kSwitch) {
        const double t0 = bessel_norm_series(g.nu, x);
        const double t1 = bessel_norm_series(g.nu + 1.0, x);   // Tn_(nu+1)
        *T = t0;
        // x Tn'(x) = -x^2 Tn_(nu+1)(x) / (2 (nu + 1))
        *D = t0 - x * x * t1 / (2.0 * (g.nu + 1.0) * (1.0 + g.b));
        return;
    }
    const cd e = std::exp(cd(0.0, x));
    const double j0 = (e * hankel_amp(g.nu, cd(x, 0.0))).real();
    const double j1 = (e * hankel_amp(g.nu + 1.0, cd(x, 0.0))).real();
    const double xp = std::pow(x, -g.nu);
    *T = g.g_nu * xp * j0;
    *D = g.g_nu * xp * (j0 - x * j1 / (1.0 + g.b));
}

// The same factors' non-oscillating Hankel parts at complex x (Z = e^{ix} P)
void transfer_amp(const Bg& g, cd x, cd* PT, cd* PD) {
    const cd xp = std::pow(x, -g.nu);
    const cd h0 = hankel_amp(g.nu, x), h1 = hankel_amp(g.nu + 1.0, x);
    *PT = g.g_nu * xp * h0;
    *PD = g.g_nu * xp * (h0 - x * h1 / (1.0 + g.b));
}

// Gauss-Legendre nodes/weights on [-1, 1] (Newton on P_n)
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& wt) {
    x.assign(n, 0.0);
    wt.assign(n, 0.0);
    for (int i = 0; i < n; ++i) {
        double z = std::cos(kPi * (i + 0.75) / (n + 0.5));
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = 0.0;
            for (int j = 1; j <= n; ++j) {
                const double p2 = p1;
                p1 = p0;
                p0 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p2) / j;
            }
            const double dp = n * (z * p0 - p1) / (z * z - 1.0);
            const double dz = p0 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) {
                x[i] = z;
                wt[i] = 2.0 / ((1.0 - z * z) * dp * dp);
                break;
            }
        }
    }
}

}  // namespace

void eos_kernel_matrices(double w, const double* c, int n, const unsigned char* pairs, double* Is, double* Ic) {
    if (!(w > 0.0 && w < 1.0)) throw std::invalid_argument("w must lie in (0, 1)");
    const Bg g = background(w);
    const double sw = std::sqrt(w);
    std::vector<double> al(n);
    double amin = 1e300;
    for (int i = 0; i < n; ++i) {
        al[i] = sw * c[i];
        amin = std::min(amin, al[i]);
    }
    const double panel = 0.25;
    if (!(amin * 2.0e4 >= kTail)) throw std::invalid_argument("sqrt(w) u_min too small for the time integrals");
    const double T1 = panel * std::ceil(kTail / amin / panel);
    // ---- nodes on [0, T1]: panels of width 0.25, 16 points, the first panel
    // split geometrically towards 0
    std::vector<double> gx, gw;
    gauss_legendre(16, gx, gw);
    std::vector<double> edges{0.0};
    for (int k = 30; k >= 1; --k) edges.push_back(panel * std::ldexp(1.0, -k));
    for (double e = panel; e < T1 + 0.5 * panel; e += panel) edges.push_back(e);
    std::vector<double> t, wt;
    for (size_t p = 0; p + 1 < edges.size(); ++p) {
        const double a = edges[p], bb = edges[p + 1];
        for (int q = 0; q < 16; ++q) {
            t.push_back(0.5 * (bb - a) * gx[q] + 0.5 * (bb + a));
            wt.push_back(0.5 * (bb - a) * gw[q]);
        }
    }
    const size_t K = t.size();
    // ---- weights t^(2(1+b)) y_m(t): y2 from its series / expansion, y1 from
    // its expansion above kSwitch and its ODE below
    std::vector<double> wy2(K), wy1(K);
    const double ymu = std::sqrt(kPi / 2.0);
    // y1(t) = -sqrt(pi/2) t^-mu Y_mu(t) with Y = Im H1; y1'(t) = sqrt(pi/2) t^-mu Y_(mu+1)(t)
    auto y_asym = [&](double tt, double* y1, double* y1d, double* y2) {
        const cd e = std::exp(cd(0.0, tt));
        const cd h0 = e * hankel_amp(g.mu, cd(tt, 0.0)), h1 = e * hankel_amp(g.mu + 1.0, cd(tt, 0.0));
        const double tp = ymu * std::pow(tt, -g.mu);
        *y1 = -tp * h0.imag();
        *y1d = tp * h1.imag();
        *y2 = tp * h0.real();
    };
    std::vector<size_t> small;
    for (size_t k = 0; k < K; ++k) {
        double y1 = 0.0, y1d = 0.0, y2 = 0.0;
        if (t[k] >= kSwitch) {
            y_asym(t[k], &y1, &y1d, &y2);
        } else {
            // t^-mu J_mu(t) = series / (Gamma(mu + 1) 2^mu)
            y2 = ymu * bessel_norm_series(g.mu, t[k]) / (std::tgamma(g.mu + 1.0) * std::pow(2.0, g.mu));
            small.push_back(k);
        }
        const double pw = std::pow(t[k], 2.0 * (1.0 + g.b));
        wy2[k] = wt[k] * pw * y2;
        wy1[k] = wt[k] * pw * y1;
    }
    {
        // RK4 in s = ln t on Y = (y, dy/ds): Y' = (y_s, -(1 + 2b) y_s - e^{2s} y)
        double y1 = 0.0, y1d = 0.0, y2 = 0.0;
        y_asym(kSwitch, &y1, &y1d, &y2);
        double s = std::log(kSwitch), y = y1, ys = kSwitch * y1d;
        const double hmax = 5e-4;
        auto rhs = [&](double ss, double a, double as, double* da, double* das) {
            *da = as;
            *das = -(1.0 + 2.0 * g.b) * as - std::exp(2.0 * ss) * a;
        };
        std::sort(small.begin(), small.end(), [&](size_t a, size_t b) { return t[a] > t[b]; });
        for (size_t k : small) {
            const double target = std::log(t[k]);
            while (s > target) {
                const double h = -std::min(hmax, s - target);
                double k1a, k1b, k2a, k2b, k3a, k3b, k4a, k4b;
                rhs(s, y, ys, &k1a, &k1b);
                rhs(s + 0.5 * h, y + 0.5 * h * k1a, ys + 0.5 * h * k1b, &k2a, &k2b);
                rhs(s + 0.5 * h, y + 0.5 * h * k2a, ys + 0.5 * h * k2b, &k3a, &k3b);
                rhs(s + h, y + h * k3a, ys + h * k3b, &k4a, &k4b);
                y += h / 6.0 * (k1a + 2.0 * k2a + 2.0 * k3a + k4a);
                ys += h / 6.0 * (k1b + 2.0 * k2b + 2.0 * k3b + k4b);
                s += h;
            }
            wy1[k] = wt[k] * std::pow(t[k], 2.0 * (1.0 + g.b)) * y;
        }
    }
    // ---- the factors at every (node, point), node-major
    std::vector<double> TT(K * size_t(n)), DD(K * size_t(n));
    for (size_t k = 0; k < K; ++k)
        for (int i = 0; i < n; ++i) transfer_pair(g, al[i] * t[k], &TT[k * n + i], &DD[k * n + i]);
    // ---- finite part on the listed pairs i <= j
    std::vector<int> pi, pj;
    for (int i = 0; i < n; ++i)
        for (int j = i; j < n; ++j)
            if (pairs[size_t(i) * n + j]) {
                pi.push_back(i);
                pj.push_back(j);
            }
    const size_t NP = pi.size();
    std::vector<double> fs(NP, 0.0), fc(NP, 0.0);
    for (size_t k = 0; k < K; ++k) {
        const double* Tk = &TT[k * n];
        const double* Dk = &DD[k * n];
        for (size_t q = 0; q < NP; ++q) {
            const double f = Tk[pi[q]] * Tk[pj[q]] + g.csrc * Dk[pi[q]] * Dk[pj[q]];
            fs[q] += wy2[k] * f;
            fc[q] += wy1[k] * f;
        }
    }
    // ---- tail: rays T1 +- i s, exp-sinh rule s = exp(pi/2 sinh x), h = 1/32
    double om_min = 1e300;
    for (size_t q = 0; q < NP; ++q)
        for (int sa = -1; sa <= 1; sa += 2)
            for (int sb = -1; sb <= 1; sb += 2)
                om_min = std::min(om_min, std::fabs(1.0 + sa * al[pi[q]] + sb * al[pj[q]]));
    if (!(om_min > 0.0)) throw std::domain_error("a point pair sits on the resonance");
    std::vector<double> sn, sw_;
    for (double x = -4.0; x <= 4.0 + 1e-12; x += 1.0 / 32.0) {
        const double s = std::exp(0.5 * kPi * std::sinh(x));
        if (s * om_min > 745.0) break;
        sn.push_back(s);
        sw_.push_back((1.0 / 32.0) * 0.5 * kPi * std::cosh(x) * s);
    }
    const size_t NS = sn.size();
    std::vector<cd> PTu(NS * n), PDu(NS * n), PTd(NS * n), PDd(NS * n), Yu(NS), Yd(NS);
    for (size_t m = 0; m < NS; ++m) {
        const cd zu(T1, sn[m]), zd(T1, -sn[m]);
        for (int i = 0; i < n; ++i) {
            transfer_amp(g, al[i] * zu, &PTu[m * n + i], &PDu[m * n + i]);
            transfer_amp(g, al[i] * zd, &PTd[m * n + i], &PDd[m * n + i]);
        }
        // y2 = Re Z, Z = sqrt(pi/2) t^-mu H1_mu(t), times the weight t^(2(1+b))
        Yu[m] = ymu * std::pow(zu, -g.mu) * hankel_amp(g.mu, zu) * std::pow(zu, 2.0 * (1.0 + g.b));
        Yd[m] = ymu * std::pow(zd, -g.mu) * hankel_amp(g.mu, zd) * std::pow(zd, 2.0 * (1.0 + g.b));
    }
    for (size_t q = 0; q < NP; ++q) {
        const int i = pi[q], j = pj[q];
        cd tail = 0.0;
        for (int sa = -1; sa <= 1; sa += 2)
            for (int sb = -1; sb <= 1; sb += 2) {
                const double om = 1.0 + sa * al[i] + sb * al[j];
                const bool up = om > 0.0;
                cd acc = 0.0;
                for (size_t m = 0; m < NS; ++m) {
                    const double x = std::fabs(om) * sn[m];
                    if (x >= 745.0) break;
                    // factor at z: P(alpha z) for sign +, conj(P(alpha conj z)) for sign -
                    const cd* PTz = up ? &PTu[m * n] : &PTd[m * n];
                    const cd* PDz = up ? &PDu[m * n] : &PDd[m * n];
                    const cd* PTc = up ? &PTd[m * n] : &PTu[m * n];
                    const cd* PDc = up ? &PDd[m * n] : &PDu[m * n];
                    const cd Ta = sa > 0 ? PTz[i] : std::conj(PTc[i]);
                    const cd Tb = sb > 0 ? PTz[j] : std::conj(PTc[j]);
                    const cd Da = sa > 0 ? PDz[i] : std::conj(PDc[i]);
                    const cd Db = sb > 0 ? PDz[j] : std::conj(PDc[j]);
                    acc += sw_[m] * std::exp(-x) * (up ? Yu[m] : Yd[m]) * (Ta * Tb + g.csrc * Da * Db);
                }
                tail += std::exp(cd(0.0, om * T1)) * (up ? cd(0.0, 1.0) : cd(0.0, -1.0)) * acc;
            }
        // y2 = Re Z_y, y1 = Re(i Z_y): the product of three real parts is 1/4 Re of the four terms
        const double s_val = fs[q] + 0.25 * tail.real();
        const double c_val = fc[q] + 0.25 * (cd(0.0, 1.0) * tail).real();
        const double r2 = g.r * g.r;
        Is[size_t(i) * n + j] = Is[size_t(j) * n + i] = r2 * s_val;
        Ic[size_t(i) * n + j] = Ic[size_t(j) * n + i] = r2 * c_val;
    }
}

}  // namespace sigw
