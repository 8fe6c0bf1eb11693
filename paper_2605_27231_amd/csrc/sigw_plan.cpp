// Host side of the C ABI: argument validation, the separable kernel tables of
// Sec. V (u-grid, kernel matrix, symmetric eigen-decomposition), plan memory,
// and the enqueue order of the per-target kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <numeric>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/sigw.h"
#include "sigw_engine.hpp"
#include "sigw_eos.hpp"

namespace {

constexpr double kPi = 3.14159265358979323846;

const char* g_noalloc_err_text();   // text of the last failed sigw_spectrum_noalloc call of this thread

bool supported_N(int N) {
    switch (N) {
        case 8: case 16: case 32: case 64: case 128: case 256: case 384: case 512: return true;
        default: return false;
    }
}

// ---------------------------------------------------------------------------
// Sec. V, Eq. grid_density: cumulative of rho(u) = 1 + A_p exp(-(u-u_p)^2/(2 sigma_p^2)).
// ---------------------------------------------------------------------------
double grid_cumulative(double u, const sigw_plan_desc& d) {
    const double s2 = std::sqrt(2.0) * d.sigma_p;
    return (u - d.u_min) + d.A_p * d.sigma_p * std::sqrt(kPi / 2.0) *
                               (std::erf((u - d.u_p) / s2) - std::erf((d.u_min - d.u_p) / s2));
}

// Edges e_n = n^{-1}(n), n = 0..n_modes: each is the smallest double where the
// normalised cumulative reaches n (bisection down to adjacent doubles).
std::vector<double> grid_edges(const sigw_plan_desc& d) {
    const int M = d.n_modes;
    std::vector<double> e(M + 1);
    const double total = grid_cumulative(d.u_max, d);
    e[0] = d.u_min;
    e[M] = d.u_max;
    for (int n = 1; n < M; ++n) {
        const double target = total * n / M;
        double lo = d.u_min, hi = d.u_max;
        for (;;) {
            const double mid = 0.5 * (lo + hi);
            if (mid <= lo || mid >= hi) break;
            if (grid_cumulative(mid, d) < target) lo = mid;
            else hi = mid;
        }
        e[n] = hi;
    }
    return e;
}

// Eq. kernels.
double kernel_s(double u, double v) {
    const double a = u * u + v * v - 3.0;
    if (!(u + v > std::sqrt(3.0))) return 0.0;
    return 27.0 * kPi * a * a / (32.0 * u * u * u * v * v * v);
}
double kernel_c(double u, double v) {
    const double a = u * u + v * v - 3.0;
    const double lg = std::log(std::fabs((3.0 - (u + v) * (u + v)) / (3.0 - (u - v) * (u - v))));
    return 27.0 * a / (32.0 * u * u * u * v * v * v) * (-4.0 * u * v + a * lg);
}

// Cyclic Jacobi eigen-decomposition of a symmetric n x n matrix (row-major).
// On return A's diagonal holds the eigenvalues and V's columns the eigenvectors.
void jacobi_eigen(std::vector<double>& A, std::vector<double>& V, int n) {
    V.assign(size_t(n) * n, 0.0);
    for (int i = 0; i < n; ++i) V[size_t(i) * n + i] = 1.0;
    auto a = [&](int i, int j) -> double& { return A[size_t(i) * n + j]; };
    auto v = [&](int i, int j) -> double& { return V[size_t(i) * n + j]; };
    double norm2 = 0.0;
    for (size_t i = 0; i < A.size(); ++i) norm2 += A[i] * A[i];
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) off += a(p, q) * a(p, q);
        if (off <= 1e-34 * norm2) break;
        for (int p = 0; p < n; ++p) {
            for (int q = p + 1; q < n; ++q) {
                const double apq = a(p, q);
                if (apq == 0.0) continue;
                const double app = a(p, p), aqq = a(q, q);
                if (std::fabs(apq) < 1e-300) {
                    a(p, q) = a(q, p) = 0.0;
                    continue;
                }
                // rotation that zeroes A_pq: t = tan(phi), the smaller root of t^2 + 2 theta t - 1 = 0
                const double theta = (aqq - app) / (2.0 * apq);
                double t = 1.0 / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                if (theta < 0.0) t = -t;
                const double c = 1.0 / std::sqrt(t * t + 1.0);
                const double s = t * c;
                const double tau = s / (1.0 + c);
                a(p, p) = app - t * apq;
                a(q, q) = aqq + t * apq;
                a(p, q) = a(q, p) = 0.0;
                for (int r = 0; r < n; ++r) {
                    if (r == p || r == q) continue;
                    const double g = a(r, p), h = a(r, q);
                    a(r, p) = a(p, r) = g - s * (h + g * tau);
                    a(r, q) = a(q, r) = h + s * (g - h * tau);
                }
                for (int r = 0; r < n; ++r) {
                    const double g = v(r, p), h = v(r, q);
                    v(r, p) = g - s * (h + g * tau);
                    v(r, q) = h + s * (g - h * tau);
                }
            }
        }
    }
}

struct Table {
    std::vector<double> sigma;   // n_alpha
    std::vector<double> phi;     // n_modes x n_alpha
};

// Sec. V: the kernel matrix C (n_modes x n_modes, row-major) diagonalised;
// the n_alpha terms of largest |sigma| are kept with their signs;
// phi_a = q_a,i / sqrt(L_i).
Table decompose_matrix(const sigw_plan_desc& d, const std::vector<double>& e, std::vector<double> A) {
    const int M = d.n_modes;
    std::vector<double> L(M);
    for (int i = 0; i < M; ++i) L[i] = e[i + 1] - e[i];
    std::vector<double> V;
    jacobi_eigen(A, V, M);
    std::vector<int> order(M);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        return std::fabs(A[size_t(x) * M + x]) > std::fabs(A[size_t(y) * M + y]);
    });
    Table t;
    t.sigma.resize(d.n_alpha);
    t.phi.assign(size_t(M) * d.n_alpha, 0.0);
    for (int a = 0; a < d.n_alpha; ++a) {
        const int k = order[a];
        t.sigma[a] = A[size_t(k) * M + k];
        for (int i = 0; i < M; ++i) t.phi[size_t(i) * d.n_alpha + a] = V[size_t(i) * M + k] / std::sqrt(L[i]);
    }
    return t;
}

// Interval centres c_i and the strip mask |c_i - c_j| <= 1 <= c_i + c_j (the
// triangle that u, v and the unit k close, Sec. V)
void centres_and_strip(const sigw_plan_desc& d, const std::vector<double>& e, std::vector<double>& c,
                       std::vector<unsigned char>& strip) {
    const int M = d.n_modes;
    c.resize(M);
    for (int i = 0; i < M; ++i) c[i] = 0.5 * (e[i] + e[i + 1]);
    strip.assign(size_t(M) * M, 0);
    for (int i = 0; i < M; ++i)
        for (int j = 0; j < M; ++j) strip[size_t(i) * M + j] = std::fabs(c[i] - c[j]) <= 1.0 && c[i] + c[j] >= 1.0;
}

// Sec. V: C_ij = sqrt(L_i L_j) I(c_i, c_j) on the strip (Eq. C_matrix_discrete)
// with the radiation-era kernels of Eq. kernels, decomposed.
Table build_table(const sigw_plan_desc& d, const std::vector<double>& e, int m) {
    const int M = d.n_modes;
    std::vector<double> c;
    std::vector<unsigned char> strip;
    centres_and_strip(d, e, c, strip);
    std::vector<double> A(size_t(M) * M, 0.0);
    for (int i = 0; i < M; ++i)
        for (int j = 0; j < M; ++j)
            if (strip[size_t(i) * M + j])
                A[size_t(i) * M + j] = std::sqrt((e[i + 1] - e[i]) * (e[j + 1] - e[j])) *
                                       (m == 0 ? kernel_s(c[i], c[j]) : kernel_c(c[i], c[j]));
    return decompose_matrix(d, e, std::move(A));
}

// The same with the kernels of a constant equation of state w (sigw_eos.cpp):
// both tables from one evaluation of the time integrals on the strip.
void build_tables_w(const sigw_plan_desc& d, const std::vector<double>& e, double w, Table out[2]) {
    const int M = d.n_modes;
    std::vector<double> c;
    std::vector<unsigned char> strip;
    centres_and_strip(d, e, c, strip);
    std::vector<double> Is(size_t(M) * M, 0.0), Ic(size_t(M) * M, 0.0);
    sigw::eos_kernel_matrices(w, c.data(), M, strip.data(), Is.data(), Ic.data());
    for (int m = 0; m < 2; ++m) {
        std::vector<double> A(size_t(M) * M, 0.0);
        const std::vector<double>& I = m == 0 ? Is : Ic;
        for (int i = 0; i < M; ++i)
            for (int j = 0; j < M; ++j)
                if (strip[size_t(i) * M + j])
                    A[size_t(i) * M + j] = std::sqrt((e[i + 1] - e[i]) * (e[j + 1] - e[j])) * I[size_t(i) * M + j];
        out[m] = decompose_matrix(d, e, std::move(A));
    }
}

// The tables depend only on the decomposition meta-parameters, and building
// them (two 200 x 200 eigen-decompositions) costs about half a second: plans
// created later in the process with the same parameters reuse them.
struct Decomposition {
    std::vector<double> edges;
    Table tab[2];
};
using DecompKey = std::tuple<int, int, double, double, double, double, double>;
std::mutex g_decomp_mu;
std::map<DecompKey, std::shared_ptr<const Decomposition>> g_decomp;

std::shared_ptr<const Decomposition> decomposition_of(const sigw_plan_desc& d) {
    const DecompKey key{d.n_modes, d.n_alpha, d.u_min, d.u_max, d.u_p, d.sigma_p, d.A_p};
    {
        std::lock_guard<std::mutex> lk(g_decomp_mu);
        auto it = g_decomp.find(key);
        if (it != g_decomp.end()) return it->second;
    }
    auto dec = std::make_shared<Decomposition>();
    dec->edges = grid_edges(d);
    for (int m = 0; m < 2; ++m) dec->tab[m] = build_table(d, dec->edges, m);
    std::lock_guard<std::mutex> lk(g_decomp_mu);
    return g_decomp.emplace(key, std::move(dec)).first->second;
}

// Constant-w tables, built once per (meta-parameters, w) in the process: the
// time integrals take seconds.
using DecompKeyW = std::tuple<int, int, double, double, double, double, double, double>;
std::map<DecompKeyW, std::shared_ptr<const Decomposition>> g_decomp_w;

std::shared_ptr<const Decomposition> decomposition_w_of(const sigw_plan_desc& d, double w) {
    const DecompKeyW key{d.n_modes, d.n_alpha, d.u_min, d.u_max, d.u_p, d.sigma_p, d.A_p, w};
    {
        std::lock_guard<std::mutex> lk(g_decomp_mu);
        auto it = g_decomp_w.find(key);
        if (it != g_decomp_w.end()) return it->second;
    }
    auto dec = std::make_shared<Decomposition>();
    dec->edges = grid_edges(d);
    build_tables_w(d, dec->edges, w, dec->tab);
    std::lock_guard<std::mutex> lk(g_decomp_mu);
    return g_decomp_w.emplace(key, std::move(dec)).first->second;
}

const char* validate(const sigw_plan_desc* d) {
    if (!d) return "NULL plan description";
    if (!supported_N(d->N)) return "N must be one of 8, 16, 32, 64, 128, 256, 384, 512";
    if (!(d->L > 0.0) || !std::isfinite(d->L)) return "L must be positive and finite";
    if (d->prec != SIGW_F32 && d->prec != SIGW_F64) return "prec must be SIGW_F32 or SIGW_F64";
    if (d->n_slots < 1 || d->n_slots > 4096) return "n_slots must be in [1, 4096]";
    if (d->n_modes < 2 || d->n_modes > 4096) return "n_modes must be in [2, 4096]";
    if (d->n_alpha < 1 || d->n_alpha > d->n_modes) return "n_alpha must be in [1, n_modes]";
    if (!(d->u_min > 0.0) || !(d->u_max > d->u_min) || !std::isfinite(d->u_max))
        return "need 0 < u_min < u_max";
    if (!(d->sigma_p > 0.0) || !(d->A_p >= 0.0) || !std::isfinite(d->u_p)) return "need sigma_p > 0, A_p >= 0";
    if (d->alpha_chunk < 0 || d->alpha_chunk > d->n_alpha) return "alpha_chunk must be in [0, n_alpha]";
    if (d->scratch_terms < 0 || d->scratch_terms > d->n_alpha) return "scratch_terms must be in [0, n_alpha]";
    if (d->batch < 0 || d->batch > 4096) return "batch must be in [0, 4096]";
    if (d->autotune != 0 && d->autotune != 1) return "autotune must be 0 or 1";
    return nullptr;
}

struct Sizes {
    long H, FS, R3, n2max;
    size_t cb, rb;
    int chunk;     // terms per xprod pass (workspace T holds 3 * chunk fields)
    int stage;     // terms staged per gen_z / ypass3 pair (scratch holds 2 * stage fields)
    int batch;     // realisations per launch (each has its own S, T and Q workspace)
};

// Default staging: every term of a pass at once when the (W, Z) pairs fit in
// 16 GiB (Phi_hat is then read once per kernel and target), else as many
// terms as fit.
constexpr size_t kStageBudget = size_t(16) << 30;

Sizes sizes_of(const sigw_plan_desc& d) {
    Sizes z;
    z.H = d.N / 2 + 1;
    z.FS = z.H * d.N * long(d.N);
    z.R3 = long(d.N) * d.N * d.N;
    z.n2max = 3L * (d.N / 2) * (d.N / 2);
    z.rb = d.prec == SIGW_F64 ? 8 : 4;
    z.cb = 2 * z.rb;
    z.chunk = d.alpha_chunk == 0 ? d.n_alpha : d.alpha_chunk;
    z.batch = d.batch == 0 ? 1 : d.batch;
    if (d.scratch_terms > 0) {
        z.stage = std::min(d.scratch_terms, z.chunk);
    } else {
        const size_t per = size_t(2) * z.FS * z.cb;
        z.stage = int(std::max<size_t>(1, std::min<size_t>(kStageBudget / per, size_t(z.chunk))));
    }
    return z;
}

constexpr int kMaxTargets = 4096;
// lattice sizes the kernels are compiled for
constexpr int kGridSizes[] = {8, 16, 32, 64, 128, 256, 384, 512};
constexpr int kSumsqBlocks = 1024;

size_t footprint_of(const sigw_plan_desc& d) {
    const Sizes z = sizes_of(d);
    const int zb = int(z.H * d.N);   // upper bound on zbin partials
    size_t b = 0;
    b += size_t(d.N) * z.cb;                                   // twiddles
    b += size_t(d.n_modes + 1) * 8;                            // edges
    b += 2 * size_t(d.n_modes) * d.n_alpha * z.rb + 2 * size_t(d.n_alpha) * z.rb;
    b += size_t(z.n2max + 1) * (2 + 1 + 8);                    // lut_u, lut_shell, amp
    b += size_t(d.n_slots) * z.FS * z.cb;                      // Phi_hat per slot
    b += size_t(z.batch) * 3 * z.chunk * z.FS * z.cb;          // gradient-field workspace
    b += size_t(z.batch) * 2 * z.stage * z.FS * z.cb;          // staged (W, Z) pairs
    b += size_t(z.batch) * 12 * z.FS * z.cb;                   // Q components (both kernels)
    b += size_t(z.R3) * z.rb;                                  // real scratch
    b += size_t(z.batch) * zb * 16 + size_t(kSumsqBlocks + 1) * 8;   // partials
    b += size_t(kMaxTargets) * (16 + 4);                       // per-target sums, slot list
    long fs_c = 0;                                             // coarse grids: twiddles, Phi_hat copies
    for (int m : kGridSizes)
        if (m < d.N) {
            b += size_t(m) * z.cb;
            fs_c = long(m / 2 + 1) * m * m;
        }
    b += size_t(z.batch) * (size_t(fs_c) * z.cb + 4);
    return b;
}

const char* kTimedNames[] = {"gen_z", "ypass", "xprod", "ypass_q", "zbin"};
constexpr int kNumTimed = 5;

}  // namespace

struct sigw_plan {
    sigw_plan_desc d{};
    Sizes z{};
    hipStream_t stream = nullptr;
    int device = 0;
    std::unique_ptr<sigw::Engine> eng;
    // smaller grids of the same box, for targets whose convolution one of
    // them computes exactly (increasing size, all below d.N)
    struct Coarse {
        int N = 0;
        void* tw = nullptr;
        std::unique_ptr<sigw::Engine> eng;
    };
    std::vector<Coarse> coarse;
    void* phi_c = nullptr;      // batch x half spectrum of the largest coarse grid
    int* d_iota = nullptr;      // 0, 1, ..., batch - 1
    std::string err;
    std::string schedule;       // report of the active x-pass schedule
    std::vector<double> edges_h;
    Table tab_h[2];
    std::vector<uint8_t> lattice_n2;   // |n|^2 values that some lattice mode has
    int grid_gen = 0;                  // bumped whenever the u grid (edges_h) changes
    // device buffers
    void* tw = nullptr;
    double* edges = nullptr;
    void* phi_tab[2] = {nullptr, nullptr};
    void* sigma_tab[2] = {nullptr, nullptr};
    int16_t* lut_u = nullptr;
    uint8_t* lut_shell = nullptr;
    double* amp = nullptr;
    void* phi_hat = nullptr;
    void* T = nullptr;
    void* Sst = nullptr;
    void* Q = nullptr;
    void* real = nullptr;
    double* part_sum = nullptr;
    unsigned long long* part_cnt = nullptr;
    double* sq_part = nullptr;
    double* sums = nullptr;
    unsigned long long* cnts = nullptr;
    // pinned host staging: results, and the spectral amplitude table of the
    // last field generation (guarded by amp_ev until its copy has run)
    double* h_amp = nullptr;
    hipEvent_t amp_ev = nullptr;
    bool amp_inflight = false;
    int* h_sel = nullptr;       // staged slot list of the last enqueued spectrum
    int* d_sel = nullptr;
    hipEvent_t sel_ev = nullptr;
    bool sel_inflight = false;
    double* h_sums = nullptr;
    unsigned long long* h_cnts = nullptr;
    std::vector<char> has_field;
    // async spectrum state
    hipEvent_t done_ev = nullptr;
    bool pending = false;
    std::vector<double> pend_targets;
    std::vector<int> pend_valid;
    // timing
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    std::vector<std::pair<int, size_t>> ev_marks;   // (kernel id, start event index)
    double t_sum[kNumTimed] = {0, 0, 0, 0, 0};
    long t_cnt[kNumTimed] = {0, 0, 0, 0, 0};
};

namespace {

sigw_status fail(sigw_plan* p, sigw_status s, const std::string& msg) {
    if (p) p->err = msg;
    return s;
}

#define HIP_TRY(p, call)                                                                    \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail((p), SIGW_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

char* cplx_at(void* base, long elems, size_t cb) { return static_cast<char*>(base) + size_t(elems) * cb; }

// Event-bracketed launch when timing is on.
template <typename F> sigw_status timed(sigw_plan* p, int id, F&& launch) {
    if (!p->timing) {
        launch();
        return SIGW_OK;
    }
    while (p->ev_pool.size() < p->ev_used + 2) {
        hipEvent_t e;
        HIP_TRY(p, hipEventCreate(&e));
        p->ev_pool.push_back(e);
    }
    const size_t i0 = p->ev_used;
    HIP_TRY(p, hipEventRecord(p->ev_pool[i0], p->stream));
    launch();
    HIP_TRY(p, hipEventRecord(p->ev_pool[i0 + 1], p->stream));
    p->ev_used += 2;
    p->ev_marks.push_back({id, i0});
    return SIGW_OK;
}

// After the stream is synchronised: fold the bracketed times into the totals.
sigw_status collect_times(sigw_plan* p) {
    for (auto& m : p->ev_marks) {
        float ms = 0.f;
        HIP_TRY(p, hipEventElapsedTime(&ms, p->ev_pool[m.second], p->ev_pool[m.second + 1]));
        p->t_sum[m.first] += ms;
        p->t_cnt[m.first] += 1;
    }
    p->ev_marks.clear();
    p->ev_used = 0;
    return SIGW_OK;
}

// Integer |n|^2 range of the shell k_lo <= k_F sqrt(n2) < k_hi, n2 > 0, using
// the same FP64 expression as the device lookup table.  The scan starts just
// below max(k_lo, 0)^2 and ends just above k_hi^2, both capped at n2max
// (which also keeps the casts of huge edges in range).
bool shell_range(double kF, double lo, double hi, long n2max, int* n2_lo, int* n2_hi) {
    auto inside = [&](long n2) {
        const double k = kF * std::sqrt((double)n2);
        return n2 > 0 && k >= lo && k < hi;
    };
    if (!(hi > lo)) return false;
    const double a = std::max(lo, 0.0) / kF;
    const double a2 = a * a;
    const long start = a2 >= double(n2max) ? n2max : std::max(1L, (long)std::floor(a2) - 2);
    long first = -1;
    for (long n2 = start; n2 <= n2max; ++n2) {
        const double k = kF * std::sqrt((double)n2);
        if (k >= hi) break;
        if (inside(n2)) {
            first = n2;
            break;
        }
    }
    if (first < 0) return false;
    const double b = hi / kF;
    const double b2 = b * b;
    long last = b2 >= double(n2max) ? n2max : std::min(n2max, (long)std::ceil(b2) + 2);
    while (last >= first && !inside(last)) --last;
    if (last < first) return false;
    // every integer in [first, last] satisfies the monotone predicate
    *n2_lo = int(first);
    *n2_hi = int(last);
    return true;
}

// Which |n|^2 in [0, 3 (N/2)^2] some mode of the N^3 lattice has: sums
// nx^2 + ny^2 + nz^2 with |n_c| <= N/2 (the signed index -N/2 has |n_c| =
// N/2).  Not every integer is one (none of the form 4^a (8b + 7), and near
// the corner of the cube fewer still), so a shell can hold |n|^2 values and
// still no mode.
std::vector<uint8_t> lattice_n2_table(int N) {
    const int h = N / 2;
    const long n2max = 3L * h * h;
    std::vector<uint8_t> two(size_t(2L * h * h + 1), 0), three(size_t(n2max + 1), 0);
    for (int x = 0; x <= h; ++x)
        for (int y = 0; y <= x; ++y) two[size_t(x * x + y * y)] = 1;
    for (long s = 0; s <= 2L * h * h; ++s)
        if (two[size_t(s)])
            for (int z = 0; z <= h; ++z) three[size_t(s + long(z) * z)] = 1;
    return three;
}

// The |n|^2 range of the modes a shell holds on the plan's lattice: the
// shell's integer range trimmed to values some lattice mode has.  False when
// the shell holds no mode; such a target gives N_b = 0 and launches nothing.
bool shell_modes(const sigw_plan* p, double lo, double hi, int* n2_lo, int* n2_hi) {
    const double kF = 2.0 * kPi / p->d.L;
    int a = 0, b = -1;
    if (!shell_range(kF, lo, hi, p->z.n2max, &a, &b)) return false;
    while (a <= b && !p->lattice_n2[size_t(a)]) ++a;
    while (b >= a && !p->lattice_n2[size_t(b)]) --b;
    if (a > b) return false;
    *n2_lo = a;
    *n2_hi = b;
    return true;
}

// Support bound of the weighted fields of target k: phi_a(u) vanishes for
// u >= u_max (the last grid edge), so every mode that the interval lookup
// maps into the grid has k_F |n| / k < u_max, i.e. |n|^2 < (u_max k / k_F)^2.
// The relative margin covers the rounding of the lookup's FP64 u; a bound
// above the true one only costs pruning, never correctness.  Capped at the
// largest |n|^2 of the lattice (n2max).
int support_n2(const sigw_plan* p, double k_target, long n2max) {
    const double kF = 2.0 * kPi / p->d.L;
    const double r = p->edges_h.back() * k_target / kF;
    const double r2 = r * r * (1.0 + 1e-12) + 1.0;
    return r2 >= double(n2max) ? int(n2max) : int(r2);
}

int isqrt_floor(long v) {
    long r = long(std::sqrt(double(v)));
    while (r > 0 && r * r > v) --r;
    while ((r + 1) * (r + 1) <= v) ++r;
    return int(r);
}

// The lattice one target's convolutions run on: the plan's own, or a smaller
// grid of the same box (same k_F).  Phi_hat of member b is at phi + sel[b] FS.
struct Grid {
    sigw::Engine* e;
    int N;
    long FS, H, n2max;
    int stage;                  // terms staged per gen_z / ypass3 pair
    const void* phi;
    const int* sel;
};

Grid own_grid(sigw_plan* p, const int* sel_dev) {
    const Sizes& z = p->z;
    return Grid{p->eng.get(), p->d.N, z.FS, z.H, z.n2max, z.stage, p->phi_hat, sel_dev};
}

// Enqueue the convolutions of one target for nb realisations on grid g,
// leaving each member's 12 components after the forward y pass in its Q
// workspace (component c at c g.FS, planes [0, n_planes)).  The member
// strides of the workspaces are the plan's (a smaller grid fits inside).
sigw_status enqueue_convolutions_on(sigw_plan* p, const Grid& g, int nb, double k_target, int n_planes) {
    const sigw_plan_desc& d = p->d;
    const Sizes& z = p->z;
    const double kF = 2.0 * kPi / d.L;
    const int n2_sup = support_n2(p, k_target, g.n2max);
    const int kx_sup = std::min(int(g.H) - 1, isqrt_floor(n2_sup));
    const double V = d.L * d.L * d.L;
    const double dV = V / (double(g.N) * g.N * g.N);
    const long s_stride = long(2) * z.stage * z.FS;
    const long t_stride = long(3) * z.chunk * z.FS;
    const long q_stride = long(12) * z.FS;
    for (int m = 0; m < 2; ++m) {
        void* Qm = cplx_at(p->Q, long(m) * 6 * g.FS, z.cb);
        for (int a0 = 0; a0 < d.n_alpha; a0 += z.chunk) {
            const int na = std::min(z.chunk, d.n_alpha - a0);
            sigw_status s;
            // stage a few terms at a time: their (W, Z) pairs are expanded
            // into gradient fields before the next group is generated
            for (int as = a0; as < a0 + na; as += g.stage) {
                const int ns = std::min(g.stage, a0 + na - as);
                void* Tdst = cplx_at(p->T, long(3) * (as - a0) * g.FS, z.cb);
                s = timed(p, 0, [&] {
                    g.e->gen_z(g.phi, g.sel, nb, p->lut_u, p->phi_tab[m], d.n_alpha, as, ns, kF, 1.0 / V, p->Sst,
                               s_stride, n2_sup, p->stream);
                });
                if (s) return s;
                s = timed(p, 1, [&] {
                    g.e->ypass3(p->Sst, ns, nb, s_stride, Tdst, t_stride, kF, n2_sup, p->stream);
                });
                if (s) return s;
            }
            s = timed(p, 2, [&] {
                g.e->xprod(p->T, t_stride, nb, p->sigma_tab[m], a0, na, dV, kF, Qm, q_stride, n_planes,
                           a0 > 0 ? 1 : 0, kx_sup, p->stream);
            });
            if (s) return s;
        }
    }
    return timed(p, 3, [&] { g.e->ypass(p->Q, 12, g.FS, n_planes, -1, nb, q_stride, p->stream); });
}

sigw_status enqueue_convolutions(sigw_plan* p, const int* sel_dev, int nb, double k_target, int n_planes) {
    return enqueue_convolutions_on(p, own_grid(p, sel_dev), nb, k_target, n_planes);
}

// The smallest coarse grid that computes target k's shell sums exactly, or
// -1.  The weighted fields have |n_c| <= Rc (support bound) and the shell
// |n_c| <= Kc.  A product of two fields has |n_c| <= 2 Rc, so on an M grid
// with M > 2 Rc + Kc no product mode aliases onto a shell mode, and with
// M > 2 Kc + 1 every shell mode has its own index, off the kz = M/2 plane:
// the circular convolution on the M grid then equals the linear one on the
// shell, and so does the plan's (which needs N > 2 Rc + Kc itself: below
// that, aliasing is part of its result and no smaller grid can reproduce
// it).  The results agree up to rounding.
int coarse_grid_for(const sigw_plan* p, double k_target, int n2_hi) {
    const int Rc = isqrt_floor(support_n2(p, k_target, p->z.n2max));
    const int Kc = isqrt_floor(n2_hi);
    const long need = std::max<long>(2L * Rc + Kc + 1, 2L * Kc + 2);
    if (need >= p->d.N) return -1;
    for (size_t i = 0; i < p->coarse.size(); ++i)
        if (p->coarse[i].N >= need) return int(i);
    return -1;
}

// Stage a host slot list into the device slot list (pinned copy, no sync
// unless the previous list's copy is still pending).
sigw_status upload_sel(sigw_plan* p, const int* slots, int n) {
    if (p->sel_inflight) {
        HIP_TRY(p, hipEventSynchronize(p->sel_ev));
        p->sel_inflight = false;
    }
    std::copy(slots, slots + n, p->h_sel);
    HIP_TRY(p, hipMemcpyAsync(p->d_sel, p->h_sel, size_t(n) * 4, hipMemcpyHostToDevice, p->stream));
    HIP_TRY(p, hipEventRecord(p->sel_ev, p->stream));
    p->sel_inflight = true;
    return SIGW_OK;
}

sigw_status check_launch(sigw_plan* p) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(p, SIGW_E_DEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
    return SIGW_OK;
}

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

sigw_status check_targets(sigw_plan* p, int n_k, const double* kt, const double* lo, const double* hi) {
    if (n_k < 0 || n_k > kMaxTargets) return fail(p, SIGW_E_INVALID, "n_k must be in [0, 4096]");
    if (n_k > 0 && (!kt || !lo || !hi)) return fail(p, SIGW_E_INVALID, "NULL target or shell array");
    for (int b = 0; b < n_k; ++b) {
        if (!finite_pos(kt[b])) return fail(p, SIGW_E_INVALID, "targets must be positive and finite");
        if (!std::isfinite(lo[b]) || !std::isfinite(hi[b]) || !(hi[b] > lo[b]))
            return fail(p, SIGW_E_INVALID, "each shell needs k_lo < k_hi, both finite");
    }
    return SIGW_OK;
}

// Enqueue lut + convolutions + zbin + finalize of targets [0, n_k) for the
// n_sel realisations in slots[]; realisation i's sums land at device offset
// i * n_k + b.  Realisations run batch at a time.  valid[b] = 0 marks an
// empty shell.
sigw_status enqueue_spectrum(sigw_plan* p, const int* sel_dev, int n_sel, int n_k, const double* kt,
                             const double* lo, const double* hi, double* sums, unsigned long long* cnts,
                             std::vector<int>& valid, bool own_grid_only) {
    const sigw_plan_desc& d = p->d;
    const Sizes& z = p->z;
    const double kF = 2.0 * kPi / d.L;
    valid.assign(n_k, 0);
    for (int b = 0; b < n_k; ++b) {
        int n2_lo = 0, n2_hi = -1;
        if (!shell_modes(p, lo[b], hi[b], &n2_lo, &n2_hi)) continue;
        valid[b] = 1;
        // the plan's lattice, or the smallest grid that gives the same sums
        const int ci = own_grid_only ? -1 : coarse_grid_for(p, kt[b], n2_hi);
        const int gN = ci < 0 ? d.N : p->coarse[ci].N;
        const int kxm = std::min(gN / 2, isqrt_floor(n2_hi));
        const int n_planes = kxm + 1;
        // the tables cover the plan's |n|^2 range, which contains any smaller grid's
        p->eng->lut(kF, kt[b], lo[b], hi[b], p->edges, d.n_modes, p->lut_u, p->lut_shell, p->stream);
        for (int g0 = 0; g0 < n_sel; g0 += z.batch) {
            const int nb = std::min(z.batch, n_sel - g0);
            Grid g = own_grid(p, sel_dev + g0);
            if (ci >= 0) {
                sigw::Engine* e = p->coarse[ci].eng.get();
                const long H = gN / 2 + 1, FS = H * gN * long(gN);
                // the (W, Z) pairs of more terms fit the staging buffer on a smaller grid
                const int stage = int(std::min<long>(z.chunk, long(z.stage) * z.FS / FS));
                g = Grid{e, gN, FS, H, 3L * (gN / 2) * (gN / 2), stage, p->phi_c, p->d_iota};
                e->restrict_half(p->phi_hat, d.N, sel_dev + g0, nb, p->phi_c, p->stream);
            }
            sigw_status s = enqueue_convolutions_on(p, g, nb, kt[b], n_planes);
            if (s) return s;
            s = timed(p, 4, [&] {
                g.e->zbin(p->Q, nb, long(12) * z.FS, p->lut_shell, n2_lo, n2_hi, p->part_sum, p->part_cnt,
                          p->stream);
            });
            if (s) return s;
            g.e->finalize(p->part_sum, p->part_cnt, g.e->zbin_blocks(), nb, sums + long(g0) * n_k + b,
                          cnts + long(g0) * n_k + b, n_k, p->stream);
        }
    }
    return check_launch(p);
}

void to_omega(const sigw_plan* p, int n_k, const double* kt, const double* S, const unsigned long long* C,
              const int* valid, double* omega, int64_t* nmodes) {
    const double V = p->d.L * p->d.L * p->d.L;
    for (int b = 0; b < n_k; ++b) {
        const bool ok = valid[b] && C[b] > 0;
        // Omega_b = k^3/(48 pi^2 V N_b) * (16/k^4) S_b, the 16/k^4 from X = -+(4/k^2) Q_hat
        if (omega) omega[b] = ok ? S[b] / (3.0 * kPi * kPi * kt[b] * V * double(C[b])) : 0.0;
        if (nmodes) nmodes[b] = ok ? int64_t(C[b]) : 0;
    }
}

sigw_status check_slot(sigw_plan* p, int slot, bool need_field) {
    if (slot < 0 || slot >= p->d.n_slots) return fail(p, SIGW_E_INVALID, "slot out of range");
    if (need_field && !p->has_field[slot]) return fail(p, SIGW_E_STATE, "no field in this slot yet");
    return SIGW_OK;
}

}  // namespace

namespace {

// Process-wide choices of the x-pass schedule per (device, N, precision):
// index and report line.
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int>, std::pair<int, std::string>> g_tune;

std::string schedule_name(sigw::Engine* e, int i) {
    int tzx = 0, occ = 0;
    e->xprod_schedule_info(i, &tzx, &occ);
    char buf[64];
    std::snprintf(buf, sizeof buf, "tzx=%d occ=%d", tzx, occ);
    return buf;
}

// Time every compiled x-pass schedule on the plan's workspace and keep the
// fastest (see sigw_autotune in the header).
sigw_status tune_xprod(sigw_plan* p, int flags) {
    const auto key = std::make_tuple(p->device, p->d.N, p->d.prec);
    sigw::Engine* e = p->eng.get();
    const int n = e->xprod_schedules();
    if (!(flags & SIGW_TUNE_FORCE)) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find(key);
        if (it != g_tune.end() && it->second.first < n) {
            e->set_xprod_schedule(it->second.first);
            p->schedule = it->second.second;
            return SIGW_OK;
        }
    }
    const sigw_plan_desc& d = p->d;
    const Sizes& z = p->z;
    const double kF = 2.0 * kPi / d.L;
    const double V = d.L * d.L * d.L;
    const double dV = V / double(z.R3);
    const long t_stride = long(3) * z.chunk * z.FS;
    const long q_stride = long(12) * z.FS;
    const int na = std::min(z.chunk, d.n_alpha);
    // defined contents for the timing launches (the values do not matter)
    HIP_TRY(p, hipMemsetAsync(p->T, 0, size_t(t_stride) * z.cb, p->stream));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(p, hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(p, SIGW_E_DEVICE, "hipEventCreate failed");
    }
    std::vector<float> best(n, 0.0f);
    sigw_status st = SIGW_OK;
    for (int i = 0; i < n && st == SIGW_OK; ++i) {
        e->set_xprod_schedule(i);
        e->xprod(p->T, t_stride, 1, p->sigma_tab[0], 0, na, dV, kF, p->Q, q_stride, int(z.H), 0, int(z.H) - 1,
                     p->stream);
        for (int r = 0; r < 3 && st == SIGW_OK; ++r) {
            float ms = 0.0f;
            if (hipEventRecord(e0, p->stream) != hipSuccess) st = SIGW_E_DEVICE;
            e->xprod(p->T, t_stride, 1, p->sigma_tab[0], 0, na, dV, kF, p->Q, q_stride, int(z.H), 0, int(z.H) - 1,
                     p->stream);
            if (st == SIGW_OK && (hipEventRecord(e1, p->stream) != hipSuccess ||
                                  hipEventSynchronize(e1) != hipSuccess ||
                                  hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                st = SIGW_E_DEVICE;
            if (st == SIGW_OK && (r == 0 || ms < best[i])) best[i] = ms;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != SIGW_OK) {
        e->set_xprod_schedule(0);
        return fail(p, st, "x-pass schedule timing failed");
    }
    int pick = 0;
    for (int i = 1; i < n; ++i)
        if (best[i] < best[pick]) pick = i;
    e->set_xprod_schedule(pick);
    std::string rep = schedule_name(e, pick) + " (timed over " + std::to_string(na) + " terms:";
    for (int i = 0; i < n; ++i) {
        char buf[96];
        std::snprintf(buf, sizeof buf, " %s %.3f ms%s", schedule_name(e, i).c_str(), double(best[i]),
                      i + 1 < n ? "," : ")");
        rep += buf;
    }
    p->schedule = rep;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = {pick, rep};
    return SIGW_OK;
}

}  // namespace

extern "C" {

const char* sigw_status_string(sigw_status s) {
    switch (s) {
        case SIGW_OK: return "ok";
        case SIGW_E_INVALID: return "invalid argument";
        case SIGW_E_NOMEM: return "out of device memory";
        case SIGW_E_DEVICE: return "device error";
        case SIGW_E_UNSUPPORTED: return "unsupported";
        case SIGW_E_STATE: return "call out of order";
        case SIGW_E_PENDING: return "pending";
    }
    return "unknown status";
}

const char* sigw_last_error(sigw_plan_t p) { return p ? p->err.c_str() : g_noalloc_err_text(); }

sigw_status sigw_plan_desc_default(sigw_plan_desc* d, int32_t N, double L, int32_t prec) {
    if (!d) return SIGW_E_INVALID;
    std::memset(d, 0, sizeof(*d));
    d->N = N;
    d->L = L;
    d->prec = prec;
    d->n_slots = 1;
    d->n_modes = 200;
    d->n_alpha = 50;
    d->u_min = 1e-3;
    d->u_max = 15.0;
    d->u_p = 1.0;
    d->sigma_p = 0.5;
    d->A_p = 10.0;
    d->alpha_chunk = 0;
    d->scratch_terms = 0;
    d->batch = 0;
    d->autotune = 0;
    return SIGW_OK;
}

sigw_status sigw_plan_footprint(const sigw_plan_desc* d, size_t* bytes) {
    if (validate(d) || !bytes) return SIGW_E_INVALID;
    *bytes = footprint_of(*d);
    return SIGW_OK;
}

sigw_status sigw_kernel_table(const sigw_plan_desc* d, int32_t m, double* sigma, double* phi, double* edges) {
    if (validate(d) || (m != 0 && m != 1)) return SIGW_E_INVALID;
    try {
        const std::shared_ptr<const Decomposition> dec = decomposition_of(*d);
        if (edges) std::copy(dec->edges.begin(), dec->edges.end(), edges);
        const Table& t = dec->tab[m];
        if (sigma) std::copy(t.sigma.begin(), t.sigma.end(), sigma);
        if (phi) std::copy(t.phi.begin(), t.phi.end(), phi);
    } catch (const std::bad_alloc&) {
        return SIGW_E_NOMEM;
    }
    return SIGW_OK;
}

sigw_status sigw_kernel_table_w(const sigw_plan_desc* d, double w, int32_t m, double* sigma, double* phi,
                                double* edges) {
    if (validate(d) || (m != 0 && m != 1) || !(w > 0.0 && w < 1.0)) return SIGW_E_INVALID;
    try {
        const std::shared_ptr<const Decomposition> dec = decomposition_w_of(*d, w);
        if (edges) std::copy(dec->edges.begin(), dec->edges.end(), edges);
        const Table& t = dec->tab[m];
        for (double s : t.sigma)
            if (!std::isfinite(s)) return SIGW_E_INVALID;
        if (sigma) std::copy(t.sigma.begin(), t.sigma.end(), sigma);
        if (phi) std::copy(t.phi.begin(), t.phi.end(), phi);
    } catch (const std::bad_alloc&) {
        return SIGW_E_NOMEM;
    } catch (const std::exception&) {
        return SIGW_E_INVALID;
    }
    return SIGW_OK;
}

sigw_status sigw_shell_modes(int32_t N, double L, double k_lo, double k_hi, int32_t* n2_lo, int32_t* n2_hi,
                             int64_t* count) {
    if (!supported_N(N) || !(L > 0.0) || !std::isfinite(L) || !std::isfinite(k_lo) || !std::isfinite(k_hi) ||
        !(k_hi > k_lo) || !count)
        return SIGW_E_INVALID;
    try {
        sigw_plan P;                       // host state only: the lattice table and the box
        P.d.N = N;
        P.d.L = L;
        P.z.n2max = 3L * (N / 2) * (N / 2);
        P.lattice_n2 = lattice_n2_table(N);
        int a = 0, b = -1;
        *count = 0;
        if (!shell_modes(&P, k_lo, k_hi, &a, &b)) return SIGW_OK;
        // modes of the signed index range [-N/2, N/2) with a given square: 1 for
        // 0 and N/2, 2 for the values in between
        const int h = N / 2;
        std::vector<int64_t> one(size_t(h) * h + 1, 0), two(size_t(2) * h * h + 1, 0);
        for (int m = 0; m <= h; ++m) one[size_t(m) * m] = (m == 0 || m == h) ? 1 : 2;
        for (int x = 0; x <= h; ++x)
            for (int y = 0; y <= h; ++y) two[size_t(x * x + y * y)] += one[size_t(x) * x] * one[size_t(y) * y];
        int64_t c = 0;
        for (long s2 = 0; s2 <= 2L * h * h; ++s2) {
            if (!two[size_t(s2)]) continue;
            for (int z = 0; z <= h; ++z) {
                const long n2 = s2 + long(z) * z;
                if (n2 >= a && n2 <= b) c += two[size_t(s2)] * one[size_t(z) * z];
            }
        }
        if (n2_lo) *n2_lo = a;
        if (n2_hi) *n2_hi = b;
        *count = c;
    } catch (const std::bad_alloc&) {
        return SIGW_E_NOMEM;
    }
    return SIGW_OK;
}

sigw_status sigw_plan_set_kernel_table(sigw_plan_t p, int32_t m, const double* sigma, const double* phi,
                                       const double* edges) {
    if (!p) return SIGW_E_INVALID;
    if ((m != 0 && m != 1) || !sigma || !phi) return fail(p, SIGW_E_INVALID, "need m in {0, 1}, sigma and phi");
    const sigw_plan_desc& d = p->d;
    const size_t na = size_t(d.n_alpha), nm = size_t(d.n_modes);
    for (size_t i = 0; i < na; ++i)
        if (!std::isfinite(sigma[i])) return fail(p, SIGW_E_INVALID, "sigma must be finite");
    for (size_t i = 0; i < nm * na; ++i)
        if (!std::isfinite(phi[i])) return fail(p, SIGW_E_INVALID, "phi must be finite");
    if (edges) {
        if (!std::isfinite(edges[0]) || !(edges[0] >= 0.0))
            return fail(p, SIGW_E_INVALID, "edges must start at a finite u >= 0");
        for (size_t i = 1; i <= nm; ++i)
            if (!std::isfinite(edges[i]) || !(edges[i] > edges[i - 1]))
                return fail(p, SIGW_E_INVALID, "edges must be finite and strictly increasing");
    }
    const Sizes& z = p->z;
    std::vector<char> sh(na * z.rb), ph(nm * na * z.rb);
    for (size_t i = 0; i < na; ++i) {
        if (d.prec == SIGW_F64) reinterpret_cast<double*>(sh.data())[i] = sigma[i];
        else reinterpret_cast<float*>(sh.data())[i] = float(sigma[i]);
    }
    for (size_t i = 0; i < nm * na; ++i) {
        if (d.prec == SIGW_F64) reinterpret_cast<double*>(ph.data())[i] = phi[i];
        else reinterpret_cast<float*>(ph.data())[i] = float(phi[i]);
    }
    // work already enqueued reads the tables: let it finish first
    HIP_TRY(p, hipStreamSynchronize(p->stream));
    HIP_TRY(p, hipMemcpy(p->sigma_tab[m], sh.data(), sh.size(), hipMemcpyHostToDevice));
    HIP_TRY(p, hipMemcpy(p->phi_tab[m], ph.data(), ph.size(), hipMemcpyHostToDevice));
    p->tab_h[m].sigma.assign(sigma, sigma + na);
    p->tab_h[m].phi.assign(phi, phi + nm * na);
    if (edges) {
        HIP_TRY(p, hipMemcpy(p->edges, edges, (nm + 1) * 8, hipMemcpyHostToDevice));
        p->edges_h.assign(edges, edges + nm + 1);     // the support bound follows the new grid
        ++p->grid_gen;                                 // graphs captured on the old grid are stale
    }
    return SIGW_OK;
}

sigw_status sigw_plan_destroy(sigw_plan_t p) {
    if (!p) return SIGW_E_INVALID;
    (void)hipStreamSynchronize(p->stream);
    void* bufs[] = {p->tw, p->edges, p->phi_tab[0], p->phi_tab[1], p->sigma_tab[0], p->sigma_tab[1],
                    p->lut_u, p->lut_shell, p->amp, p->phi_hat, p->T, p->Sst, p->Q, p->real, p->part_sum,
                    p->part_cnt, p->sq_part, p->sums, p->cnts, p->d_sel};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    for (auto& c : p->coarse)
        if (c.tw) (void)hipFree(c.tw);
    if (p->phi_c) (void)hipFree(p->phi_c);
    if (p->d_iota) (void)hipFree(p->d_iota);
    if (p->h_amp) (void)hipHostFree(p->h_amp);
    if (p->amp_ev) (void)hipEventDestroy(p->amp_ev);
    if (p->h_sel) (void)hipHostFree(p->h_sel);
    if (p->sel_ev) (void)hipEventDestroy(p->sel_ev);
    if (p->h_sums) (void)hipHostFree(p->h_sums);
    if (p->h_cnts) (void)hipHostFree(p->h_cnts);
    if (p->done_ev) (void)hipEventDestroy(p->done_ev);
    for (auto e : p->ev_pool) (void)hipEventDestroy(e);
    delete p;
    return SIGW_OK;
}

sigw_status sigw_plan_create(const sigw_plan_desc* d, void* hip_stream, sigw_plan_t* out) {
    if (!out) return SIGW_E_INVALID;
    *out = nullptr;
    if (const char* why = validate(d)) {
        (void)why;
        return SIGW_E_INVALID;
    }
    std::unique_ptr<sigw_plan> p(new (std::nothrow) sigw_plan());
    if (!p) return SIGW_E_NOMEM;
    p->d = *d;
    p->z = sizes_of(*d);
    p->stream = static_cast<hipStream_t>(hip_stream);
    p->has_field.assign(d->n_slots, 0);
    try {
        p->lattice_n2 = lattice_n2_table(d->N);
    } catch (const std::bad_alloc&) {
        return SIGW_E_NOMEM;
    }
    // Sec. V tables on the host (built once per parameter set in the process)
    try {
        const std::shared_ptr<const Decomposition> dec = decomposition_of(*d);
        p->edges_h = dec->edges;
        for (int m = 0; m < 2; ++m) p->tab_h[m] = dec->tab[m];
    } catch (const std::bad_alloc&) {
        return SIGW_E_NOMEM;
    }
    for (int m = 0; m < 2; ++m)
        for (double s : p->tab_h[m].sigma)
            if (!std::isfinite(s)) return SIGW_E_INVALID;
    sigw_plan* P = p.get();
    int dev_count = 0;
    if (hipGetDeviceCount(&dev_count) != hipSuccess || dev_count < 1) return SIGW_E_DEVICE;
    if (hipGetDevice(&P->device) != hipSuccess) return SIGW_E_DEVICE;
    const Sizes& z = P->z;
    auto alloc = [&](void** ptr, size_t bytes) -> bool {
        if (hipMalloc(ptr, bytes) != hipSuccess) {
            (void)hipGetLastError();
            *ptr = nullptr;
            return false;
        }
        return true;
    };
    const long zb_max = long(z.H * d->N) * z.batch;
    bool ok = alloc(&P->tw, size_t(d->N) * z.cb) && alloc((void**)&P->edges, (d->n_modes + 1) * 8) &&
              alloc(&P->phi_tab[0], size_t(d->n_modes) * d->n_alpha * z.rb) &&
              alloc(&P->phi_tab[1], size_t(d->n_modes) * d->n_alpha * z.rb) &&
              alloc(&P->sigma_tab[0], size_t(d->n_alpha) * z.rb) && alloc(&P->sigma_tab[1], size_t(d->n_alpha) * z.rb) &&
              alloc((void**)&P->lut_u, size_t(z.n2max + 1) * 2) && alloc((void**)&P->lut_shell, size_t(z.n2max + 1)) &&
              alloc((void**)&P->amp, size_t(z.n2max + 1) * 8) &&
              alloc(&P->phi_hat, size_t(d->n_slots) * z.FS * z.cb) &&
              alloc(&P->T, size_t(z.batch) * 3 * z.chunk * z.FS * z.cb) &&
              alloc(&P->Sst, size_t(z.batch) * 2 * z.stage * z.FS * z.cb) &&
              alloc(&P->Q, size_t(z.batch) * 12 * z.FS * z.cb) && alloc((void**)&P->d_sel, size_t(kMaxTargets) * 4) &&
              alloc(&P->real, size_t(z.R3) * z.rb) && alloc((void**)&P->part_sum, size_t(zb_max) * 8) &&
              alloc((void**)&P->part_cnt, size_t(zb_max) * 8) &&
              alloc((void**)&P->sq_part, size_t(kSumsqBlocks + 1) * 8) &&
              alloc((void**)&P->sums, size_t(kMaxTargets) * 8) && alloc((void**)&P->cnts, size_t(kMaxTargets) * 8);
    if (!ok) {
        sigw_plan_destroy(p.release());
        return SIGW_E_NOMEM;
    }
    if (hipHostMalloc((void**)&P->h_sums, kMaxTargets * 8) != hipSuccess ||
        hipHostMalloc((void**)&P->h_cnts, kMaxTargets * 8) != hipSuccess ||
        hipHostMalloc((void**)&P->h_amp, size_t(z.n2max + 1) * 8) != hipSuccess ||
        hipHostMalloc((void**)&P->h_sel, size_t(kMaxTargets) * 4) != hipSuccess ||
        hipEventCreate(&P->sel_ev) != hipSuccess ||
        hipEventCreate(&P->amp_ev) != hipSuccess || hipEventCreate(&P->done_ev) != hipSuccess) {
        sigw_plan_destroy(p.release());
        return SIGW_E_DEVICE;
    }
    // tables: twiddles, edges, phi, sigma (in the path precision)
    std::vector<char> twh(size_t(d->N) * z.cb);
    sigw::host_twiddles(d->prec, d->N, twh.data());
    std::vector<char> phih[2], sigh[2];
    for (int m = 0; m < 2; ++m) {
        const Table& t = P->tab_h[m];
        phih[m].resize(t.phi.size() * z.rb);
        sigh[m].resize(t.sigma.size() * z.rb);
        for (size_t i = 0; i < t.phi.size(); ++i) {
            if (d->prec == SIGW_F64) reinterpret_cast<double*>(phih[m].data())[i] = t.phi[i];
            else reinterpret_cast<float*>(phih[m].data())[i] = (float)t.phi[i];
        }
        for (size_t i = 0; i < t.sigma.size(); ++i) {
            if (d->prec == SIGW_F64) reinterpret_cast<double*>(sigh[m].data())[i] = t.sigma[i];
            else reinterpret_cast<float*>(sigh[m].data())[i] = (float)t.sigma[i];
        }
    }
    bool up = hipMemcpy(P->tw, twh.data(), twh.size(), hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(P->edges, P->edges_h.data(), P->edges_h.size() * 8, hipMemcpyHostToDevice) == hipSuccess;
    for (int m = 0; m < 2 && up; ++m)
        up = hipMemcpy(P->phi_tab[m], phih[m].data(), phih[m].size(), hipMemcpyHostToDevice) == hipSuccess &&
             hipMemcpy(P->sigma_tab[m], sigh[m].data(), sigh[m].size(), hipMemcpyHostToDevice) == hipSuccess;
    if (!up) {
        sigw_plan_destroy(p.release());
        return SIGW_E_DEVICE;
    }
    P->eng.reset(sigw::make_engine(d->prec, d->N, P->tw));
    if (!P->eng) {
        sigw_plan_destroy(p.release());
        return SIGW_E_UNSUPPORTED;
    }
    // coarse grids: an engine and a twiddle table each, one Phi_hat copy per
    // batch member at the largest, and the member index list
    long fs_c = 0;
    for (int m : kGridSizes) {
        if (m >= d->N) break;
        sigw_plan::Coarse c;
        c.N = m;
        std::vector<char> tw(size_t(m) * z.cb);
        sigw::host_twiddles(d->prec, m, tw.data());
        if (!alloc(&c.tw, tw.size()) ||
            hipMemcpy(c.tw, tw.data(), tw.size(), hipMemcpyHostToDevice) != hipSuccess) {
            P->coarse.push_back(std::move(c));
            sigw_plan_destroy(p.release());
            return SIGW_E_NOMEM;
        }
        c.eng.reset(sigw::make_engine(d->prec, m, c.tw));
        const bool made = bool(c.eng);
        P->coarse.push_back(std::move(c));
        if (!made) {
            sigw_plan_destroy(p.release());
            return SIGW_E_UNSUPPORTED;
        }
        fs_c = long(m / 2 + 1) * m * m;
    }
    {
        std::vector<int> iota(z.batch);
        for (int i = 0; i < z.batch; ++i) iota[i] = i;
        const bool okc = (fs_c == 0 || alloc(&P->phi_c, size_t(z.batch) * fs_c * z.cb)) &&
                         alloc((void**)&P->d_iota, size_t(z.batch) * 4) &&
                         hipMemcpy(P->d_iota, iota.data(), iota.size() * 4, hipMemcpyHostToDevice) == hipSuccess;
        if (!okc) {
            sigw_plan_destroy(p.release());
            return SIGW_E_NOMEM;
        }
    }
    P->schedule = schedule_name(P->eng.get(), 0);
    if (d->autotune) {
        const sigw_status st = tune_xprod(P, 0);
        if (st != SIGW_OK) {
            sigw_plan_destroy(p.release());
            return st;
        }
    }
    *out = p.release();
    return SIGW_OK;
}

sigw_status sigw_white_noise(sigw_plan_t p, uint64_t seed, void* out_dev) {
    if (!p || !out_dev) return fail(p, SIGW_E_INVALID, "NULL argument");
    p->eng->noise(seed, out_dev, p->stream);
    return check_launch(p);
}

namespace {
// Phi_hat[slot] = dV DFT(scale * map(real)); real holds zeta_g on entry.
sigw_status finish_field(sigw_plan* p, int slot, const sigw::MapParams& mp, bool reduce) {
    const Sizes& z = p->z;
    const double V = p->d.L * p->d.L * p->d.L;
    const double dV = V / double(z.R3);
    if (reduce) p->eng->sumsq(p->real, p->sq_part, p->sq_part + kSumsqBlocks, p->stream);
    p->eng->map_scale(p->real, p->real, p->sq_part + kSumsqBlocks, mp, (2.0 / 3.0) * dV, p->stream);
    void* dst = cplx_at(p->phi_hat, long(slot) * z.FS, z.cb);
    p->eng->xpass_r2c(p->real, dst, p->stream);
    p->eng->ypass(dst, 1, z.FS, int(z.H), -1, 1, 0, p->stream);
    p->eng->zpass(dst, z.H * p->d.N, -1, p->stream);
    sigw_status s = check_launch(p);
    if (s == SIGW_OK) p->has_field[slot] = 1;
    return s;
}
}  // namespace

sigw_status sigw_generate_field(sigw_plan_t p, int32_t slot, uint64_t seed, const sigw_lognormal* sp,
                                const sigw_ngmap* mp) {
    if (!p || !sp || !mp) return fail(p, SIGW_E_INVALID, "NULL argument");
    if (sigw_status s = check_slot(p, slot, false)) return s;
    if (!(sp->A >= 0.0) || !finite_pos(sp->sigma) || !finite_pos(sp->k_star) || !std::isfinite(sp->A))
        return fail(p, SIGW_E_INVALID, "log-normal needs A >= 0, sigma > 0, k_star > 0");
    if (mp->kind < 0 || mp->kind > 3) return fail(p, SIGW_E_INVALID, "unknown map kind");
    if (mp->kind == 3 && (!finite_pos(mp->k_NL) || !std::isfinite(mp->alpha_NL) || !std::isfinite(mp->beta_NL)))
        return fail(p, SIGW_E_INVALID, "non-local map needs finite alpha_NL, beta_NL and k_NL > 0");
    if (mp->kind == 2 && (!finite_pos(mp->beta) || !finite_pos(mp->clip)))
        return fail(p, SIGW_E_INVALID, "exponential tail needs beta > 0 and clip > 0");
    if (mp->kind == 1 && (!std::isfinite(mp->F_NL) || !std::isfinite(mp->G_NL)))
        return fail(p, SIGW_E_INVALID, "local map needs finite F_NL, G_NL");
    const sigw_plan_desc& d = p->d;
    const Sizes& z = p->z;
    const double kF = 2.0 * kPi / d.L;
    const double V = d.L * d.L * d.L;
    const double dV = V / double(z.R3);
    // amplitude per |n|^2: sqrt(dV P(k_F |n|)) / V, zero at n = 0 (the 1/V is the
    // inverse-transform normalisation of zeta_g(x) = (1/V) sum exp(iqx) zeta_hat)
    if (p->amp_inflight) {
        HIP_TRY(p, hipEventSynchronize(p->amp_ev));   // the previous table's copy has run
        p->amp_inflight = false;
    }
    double* amp = p->h_amp;
    amp[0] = 0.0;
    for (long n2 = 1; n2 <= z.n2max; ++n2) {
        const double k = kF * std::sqrt((double)n2);
        const double lk = std::log(k / sp->k_star);
        const double d2 = sp->A / std::sqrt(2.0 * kPi * sp->sigma * sp->sigma) *
                          std::exp(-lk * lk / (2.0 * sp->sigma * sp->sigma));
        const double P = 2.0 * kPi * kPi * d2 / (k * k * k);
        amp[n2] = std::sqrt(dV * P) / V;
    }
    HIP_TRY(p, hipMemcpyAsync(p->amp, amp, size_t(z.n2max + 1) * 8, hipMemcpyHostToDevice, p->stream));
    HIP_TRY(p, hipEventRecord(p->amp_ev, p->stream));
    p->amp_inflight = true;
    void* half = p->Q;   // scratch half spectrum
    p->eng->noise(seed, p->real, p->stream);
    p->eng->xpass_r2c(p->real, half, p->stream);
    p->eng->ypass(half, 1, z.FS, int(z.H), -1, 1, 0, p->stream);
    p->eng->zpass(half, z.H * d.N, -1, p->stream);
    p->eng->filter(half, p->amp, p->stream);
    auto c2r = [&](void* h, void* real_out) {
        p->eng->zpass(h, z.H * d.N, +1, p->stream);
        p->eng->ypass(h, 1, z.FS, int(z.H), +1, 1, 0, p->stream);
        p->eng->xpass_c2r(h, real_out, p->stream);
    };
    if (mp->kind != 3) {
        c2r(half, p->real);
        sigw::MapParams m{mp->kind, mp->F_NL, mp->G_NL, mp->beta, mp->clip};
        return finish_field(p, slot, m, mp->kind == 1);
    }
    // Eq. nonlocal, in the gradient-field workspace: hl (half spectrum),
    // l2 = (beta_NL/k_NL^2) lap zeta_g, l1 = (alpha_NL/k_NL^2) lap(zeta_g^2)
    void* hl = p->T;
    void* l2 = cplx_at(p->T, z.FS, z.cb);
    void* l1 = cplx_at(p->T, 2 * z.FS, z.cb);
    const double c_nl = -kF * kF / (mp->k_NL * mp->k_NL);
    HIP_TRY(p, hipMemcpyAsync(hl, half, size_t(z.FS) * z.cb, hipMemcpyDeviceToDevice, p->stream));
    p->eng->laplacian(hl, mp->beta_NL * c_nl, p->stream);
    c2r(hl, l2);
    c2r(half, p->real);                                    // zeta_g
    p->eng->square(p->real, l1, p->stream);
    p->eng->xpass_r2c(l1, hl, p->stream);
    p->eng->ypass(hl, 1, z.FS, int(z.H), -1, 1, 0, p->stream);
    p->eng->zpass(hl, z.H * d.N, -1, p->stream);
    // the forward and inverse passes are unnormalised: divide by N^3
    p->eng->laplacian(hl, mp->alpha_NL * c_nl / double(z.R3), p->stream);
    c2r(hl, l1);
    p->eng->nonlocal_combine(p->real, l1, l2, p->real, p->stream);
    sigw::MapParams m{0, 0.0, 0.0, 0.0, 0.0};
    return finish_field(p, slot, m, false);
}

sigw_status sigw_set_zeta(sigw_plan_t p, int32_t slot, const void* zeta_dev) {
    if (!p || !zeta_dev) return fail(p, SIGW_E_INVALID, "NULL argument");
    if (sigw_status s = check_slot(p, slot, false)) return s;
    HIP_TRY(p, hipMemcpyAsync(p->real, zeta_dev, size_t(p->z.R3) * p->z.rb, hipMemcpyDeviceToDevice, p->stream));
    sigw::MapParams m{0, 0, 0, 0, 0};
    return finish_field(p, slot, m, false);
}

sigw_status sigw_set_phi_hat(sigw_plan_t p, int32_t slot, const void* src) {
    if (!p || !src) return fail(p, SIGW_E_INVALID, "NULL argument");
    if (sigw_status s = check_slot(p, slot, false)) return s;
    HIP_TRY(p, hipMemcpyAsync(cplx_at(p->phi_hat, long(slot) * p->z.FS, p->z.cb), src, size_t(p->z.FS) * p->z.cb,
                              hipMemcpyDeviceToDevice, p->stream));
    p->has_field[slot] = 1;
    return SIGW_OK;
}

sigw_status sigw_get_phi_hat(sigw_plan_t p, int32_t slot, void* dst) {
    if (!p || !dst) return fail(p, SIGW_E_INVALID, "NULL argument");
    if (sigw_status s = check_slot(p, slot, true)) return s;
    HIP_TRY(p, hipMemcpyAsync(dst, cplx_at(p->phi_hat, long(slot) * p->z.FS, p->z.cb), size_t(p->z.FS) * p->z.cb,
                              hipMemcpyDeviceToDevice, p->stream));
    return SIGW_OK;
}

sigw_status sigw_source_convolutions(sigw_plan_t p, int32_t slot, double k_target, void* qhat_dev) {
    if (!p || !qhat_dev) return fail(p, SIGW_E_INVALID, "NULL argument");
    if (!finite_pos(k_target)) return fail(p, SIGW_E_INVALID, "k_target must be positive");
    if (sigw_status s = check_slot(p, slot, true)) return s;
    const Sizes& z = p->z;
    const double kF = 2.0 * kPi / p->d.L;
    p->eng->lut(kF, k_target, 0.0, 0.0, p->edges, p->d.n_modes, p->lut_u, p->lut_shell, p->stream);
    if (sigw_status s = upload_sel(p, &slot, 1)) return s;
    if (sigw_status s = enqueue_convolutions(p, p->d_sel, 1, k_target, int(z.H))) return s;
    p->eng->zpass(p->Q, 12 * z.H * p->d.N, -1, p->stream);
    HIP_TRY(p, hipMemcpyAsync(qhat_dev, p->Q, size_t(12) * z.FS * z.cb, hipMemcpyDeviceToDevice, p->stream));
    return check_launch(p);
}

sigw_status sigw_spectrum_batch(sigw_plan_t p, int32_t n_sel, const int32_t* slots, int32_t n_k, const double* kt,
                                const double* lo, const double* hi, double* omega, int64_t* nmodes) {
    if (!p) return SIGW_E_INVALID;
    if (p->pending) return fail(p, SIGW_E_STATE, "an asynchronous spectrum is still in flight");
    if (n_sel < 1 || !slots) return fail(p, SIGW_E_INVALID, "need at least one slot");
    if (sigw_status s = check_targets(p, n_k, kt, lo, hi)) return s;
    if (long(n_sel) * n_k > kMaxTargets) return fail(p, SIGW_E_INVALID, "n_sel * n_k exceeds 4096");
    for (int i = 0; i < n_sel; ++i)
        if (sigw_status s = check_slot(p, slots[i], true)) return s;
    std::vector<int> valid;
    if (sigw_status s = upload_sel(p, slots, n_sel)) return s;
    if (sigw_status s = enqueue_spectrum(p, p->d_sel, n_sel, n_k, kt, lo, hi, p->sums, p->cnts, valid, false))
        return s;
    const size_t cnt = size_t(n_sel) * n_k;
    if (cnt) {
        HIP_TRY(p, hipMemcpyAsync(p->h_sums, p->sums, cnt * 8, hipMemcpyDeviceToHost, p->stream));
        HIP_TRY(p, hipMemcpyAsync(p->h_cnts, p->cnts, cnt * 8, hipMemcpyDeviceToHost, p->stream));
    }
    HIP_TRY(p, hipStreamSynchronize(p->stream));
    if (p->timing) {
        if (sigw_status s = collect_times(p)) return s;
    }
    for (int i = 0; i < n_sel; ++i)
        to_omega(p, n_k, kt, p->h_sums + i * n_k, p->h_cnts + i * n_k, valid.data(),
                 omega ? omega + size_t(i) * n_k : nullptr, nmodes ? nmodes + size_t(i) * n_k : nullptr);
    return SIGW_OK;
}

sigw_status sigw_spectrum_jackknife(sigw_plan_t p, int32_t slot, int32_t n_k, const double* kt, const double* lo,
                                    const double* hi, int32_t M, double* omega, int64_t* nmodes, double* omega_err,
                                    double* replicas) {
    if (!p) return SIGW_E_INVALID;
    if (p->pending) return fail(p, SIGW_E_STATE, "an asynchronous spectrum is still in flight");
    if (sigw_status s = check_targets(p, n_k, kt, lo, hi)) return s;
    if (sigw_status s = check_slot(p, slot, true)) return s;
    const sigw_plan_desc& d = p->d;
    const Sizes& z = p->z;
    const long M3 = long(M) * M * M;
    if (M < 2 || d.N % M != 0 || M3 >= kMaxTargets || M3 > z.H * d.N)
        return fail(p, SIGW_E_INVALID, "M must be >= 2, divide N, and M^3 stay below 4096");
    const double kF = 2.0 * kPi / d.L;
    for (int b = 0; b < n_k; ++b)
        if (hi[b] > kF * (d.N / 2)) return fail(p, SIGW_E_INVALID, "jackknife shells must lie below k_F N/2");
    // E (one FP64 value per site) lives in the gradient-field workspace,
    // which is free once the x pass of a target has run
    double* E = static_cast<double*>(p->T);
    const double wcomp[6] = {1.0, 1.0, 1.0, 2.0, 2.0, 2.0};   // off-diagonal components stand for two
    if (sigw_status s = upload_sel(p, &slot, 1)) return s;
    for (int b = 0; b < n_k; ++b) {
        std::vector<int> valid;
        // the replicas need the shell's modes on the plan's own lattice
        if (sigw_status s =
                enqueue_spectrum(p, p->d_sel, 1, 1, kt + b, lo + b, hi + b, p->sums, p->cnts, valid, true))
            return s;
        double* S_i = p->part_sum;     // after finalize has consumed the zbin partials
        if (valid[0]) {
            int n2_lo = 0, n2_hi = -1;
            shell_modes(p, lo[b], hi[b], &n2_lo, &n2_hi);
            p->eng->ztt(p->Q, p->lut_shell, n2_lo, n2_hi, p->stream);
            for (int c = 0; c < 12; ++c) {
                void* comp = cplx_at(p->Q, long(c) * z.FS, z.cb);
                p->eng->zpass(comp, z.H * d.N, +1, p->stream);
                p->eng->ypass(comp, 1, z.FS, int(z.H), +1, 1, 0, p->stream);
                p->eng->xpass_c2r(comp, p->real, p->stream);
                p->eng->energy_accum(p->real, E, wcomp[c % 6], c == 0 ? 1 : 0, p->stream);
            }
            p->eng->subvol_sums(E, M, S_i, p->stream);
            HIP_TRY(p, hipMemcpyAsync(p->h_sums + 1, S_i, size_t(M3) * 8, hipMemcpyDeviceToHost, p->stream));
        }
        HIP_TRY(p, hipMemcpyAsync(p->h_sums, p->sums, 8, hipMemcpyDeviceToHost, p->stream));
        HIP_TRY(p, hipMemcpyAsync(p->h_cnts, p->cnts, 8, hipMemcpyDeviceToHost, p->stream));
        if (sigw_status s = check_launch(p)) return s;
        HIP_TRY(p, hipStreamSynchronize(p->stream));
        double om = 0.0;
        int64_t nb = 0;
        to_omega(p, 1, kt + b, p->h_sums, p->h_cnts, valid.data(), &om, &nb);
        if (omega) omega[b] = om;
        if (nmodes) nmodes[b] = nb;
        double err = 0.0;
        if (valid[0] && nb > 0) {
            // the unnormalised inverse passes give sum_x |h|^2 = N^3 sum_n |Y|^2
            const double inv_n3 = 1.0 / double(z.R3);
            double S = 0.0;
            for (long i = 0; i < M3; ++i) S += p->h_sums[1 + i] * inv_n3;
            std::vector<double> rep(M3);
            double mean = 0.0;
            for (long i = 0; i < M3; ++i) {
                const double Si = double(M3) / double(M3 - 1) * (S - p->h_sums[1 + i] * inv_n3);
                const unsigned long long cnt = (unsigned long long)nb;
                const int ok = 1;
                to_omega(p, 1, kt + b, &Si, &cnt, &ok, &rep[i], nullptr);
                mean += rep[i];
            }
            mean /= double(M3);
            double var = 0.0;
            for (long i = 0; i < M3; ++i) var += (rep[i] - mean) * (rep[i] - mean);
            err = std::sqrt(double(M3 - 1) / double(M3) * var);
            if (replicas) std::copy(rep.begin(), rep.end(), replicas + size_t(b) * M3);
        } else if (replicas) {
            std::fill(replicas + size_t(b) * M3, replicas + size_t(b + 1) * M3, 0.0);
        }
        if (omega_err) omega_err[b] = err;
    }
    return SIGW_OK;
}

sigw_status sigw_spectrum_adaptive(sigw_plan_t p, int32_t slot, uint64_t seed, const sigw_lognormal* sp,
                                   const sigw_ngmap* mp, int32_t n_k, const double* kt, double eps, double* omega,
                                   int64_t* nmodes, double* box) {
    if (!p || !sp || !mp) return fail(p, SIGW_E_INVALID, "NULL argument");
    if (p->pending) return fail(p, SIGW_E_STATE, "an asynchronous spectrum is still in flight");
    if (sigw_status s = check_slot(p, slot, false)) return s;
    if (n_k < 0 || n_k > kMaxTargets || (n_k > 0 && !kt)) return fail(p, SIGW_E_INVALID, "bad target list");
    for (int b = 0; b < n_k; ++b)
        if (!finite_pos(kt[b])) return fail(p, SIGW_E_INVALID, "targets must be positive and finite");
    if (!(eps > 0.0 && eps < 1.0)) return fail(p, SIGW_E_INVALID, "eps must be in (0, 1)");
    if (!finite_pos(sp->sigma) || !finite_pos(sp->k_star))
        return fail(p, SIGW_E_INVALID, "log-normal needs sigma > 0, k_star > 0");
    // k_bar: Delta^2 is a normal density in log k (mean log k*, width sigma),
    // so the power fraction below k is Phi((log k - log k*)/sigma); invert
    // Phi(z) = 1 - eps by bisection
    double za = -40.0, zb = 40.0;
    for (int it = 0; it < 200; ++it) {
        const double zm = 0.5 * (za + zb);
        if (0.5 * std::erfc(-zm / std::sqrt(2.0)) < 1.0 - eps) za = zm;
        else zb = zm;
    }
    const double kbar = sp->k_star * std::exp(sp->sigma * 0.5 * (za + zb));
    const double L0 = p->d.L;
    sigw_status st = SIGW_OK;
    for (int b = 0; b < n_k && st == SIGW_OK; ++b) {
        const double L = kPi * p->d.N / (3.0 * std::max(kt[b], kbar));
        p->d.L = L;
        st = sigw_generate_field(p, slot, seed, sp, mp);
        double om = 0.0;
        int64_t nb = 0;
        if (st == SIGW_OK) {
            const double lo = kt[b] - kPi / L, hi = kt[b] + kPi / L;
            st = sigw_spectrum(p, slot, 1, kt + b, &lo, &hi, &om, &nb);
        }
        if (omega) omega[b] = om;
        if (nmodes) nmodes[b] = nb;
        if (box) box[b] = L;
    }
    // the slot now holds a field of the last target's box: it must be generated again
    p->d.L = L0;
    p->has_field[slot] = 0;
    return st;
}

sigw_status sigw_spectrum(sigw_plan_t p, int32_t slot, int32_t n_k, const double* kt, const double* lo,
                          const double* hi, double* omega, int64_t* nmodes) {
    return sigw_spectrum_batch(p, 1, &slot, n_k, kt, lo, hi, omega, nmodes);
}

sigw_status sigw_spectrum_enqueue(sigw_plan_t p, int32_t slot, int32_t n_k, const double* kt, const double* lo,
                                  const double* hi) {
    if (!p) return SIGW_E_INVALID;
    if (p->pending) return fail(p, SIGW_E_STATE, "an asynchronous spectrum is already in flight");
    if (n_k > 64) return fail(p, SIGW_E_INVALID, "asynchronous spectra take at most 64 targets");
    if (sigw_status s = check_targets(p, n_k, kt, lo, hi)) return s;
    if (sigw_status s = check_slot(p, slot, true)) return s;
    if (sigw_status s = upload_sel(p, &slot, 1)) return s;
    if (sigw_status s = enqueue_spectrum(p, p->d_sel, 1, n_k, kt, lo, hi, p->sums, p->cnts, p->pend_valid, false))
        return s;
    if (n_k) {
        HIP_TRY(p, hipMemcpyAsync(p->h_sums, p->sums, size_t(n_k) * 8, hipMemcpyDeviceToHost, p->stream));
        HIP_TRY(p, hipMemcpyAsync(p->h_cnts, p->cnts, size_t(n_k) * 8, hipMemcpyDeviceToHost, p->stream));
    }
    HIP_TRY(p, hipEventRecord(p->done_ev, p->stream));
    p->pend_targets.assign(kt, kt + n_k);
    p->pending = true;
    return SIGW_OK;
}

sigw_status sigw_spectrum_poll(sigw_plan_t p, double* omega, int64_t* nmodes) {
    if (!p) return SIGW_E_INVALID;
    if (!p->pending) return fail(p, SIGW_E_STATE, "no asynchronous spectrum in flight");
    hipError_t e = hipEventQuery(p->done_ev);
    if (e == hipErrorNotReady) return SIGW_E_PENDING;
    if (e != hipSuccess) {
        p->pending = false;
        return fail(p, SIGW_E_DEVICE, std::string("hipEventQuery: ") + hipGetErrorString(e));
    }
    p->pending = false;
    if (p->timing) {
        if (sigw_status s = collect_times(p)) return s;
    }
    const int n_k = int(p->pend_targets.size());
    to_omega(p, n_k, p->pend_targets.data(), p->h_sums, p->h_cnts, p->pend_valid.data(), omega, nmodes);
    return SIGW_OK;
}

// ---------------------------------------------------------------------------
// Captured spectra: the whole enqueue sequence of one batched spectrum as a
// HIP graph, replayed for new fields in the same slots.
// ---------------------------------------------------------------------------
}  // extern "C"

struct sigw_graph {
    sigw_plan* p = nullptr;
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    int n_sel = 0, n_k = 0;
    std::vector<double> kt;
    std::vector<int> valid;
    int grid_gen = 0;           // the plan's u-grid generation at capture
    int* d_slots = nullptr;
    double* d_sums = nullptr;
    unsigned long long* d_cnts = nullptr;
    double* h_sums = nullptr;
    unsigned long long* h_cnts = nullptr;
    bool launched = false;
};

extern "C" {

sigw_status sigw_graph_destroy(sigw_graph_t gr) {
    if (!gr) return SIGW_E_INVALID;
    if (gr->p) (void)hipStreamSynchronize(gr->p->stream);
    if (gr->ge) (void)hipGraphExecDestroy(gr->ge);
    if (gr->g) (void)hipGraphDestroy(gr->g);
    if (gr->d_slots) (void)hipFree(gr->d_slots);
    if (gr->d_sums) (void)hipFree(gr->d_sums);
    if (gr->d_cnts) (void)hipFree(gr->d_cnts);
    if (gr->h_sums) (void)hipHostFree(gr->h_sums);
    if (gr->h_cnts) (void)hipHostFree(gr->h_cnts);
    delete gr;
    return SIGW_OK;
}

sigw_status sigw_graph_create(sigw_plan_t p, int32_t n_sel, const int32_t* slots, int32_t n_k, const double* kt,
                              const double* lo, const double* hi, sigw_graph_t* out) {
    if (!p || !out) return SIGW_E_INVALID;
    *out = nullptr;
    if (p->pending) return fail(p, SIGW_E_STATE, "an asynchronous spectrum is still in flight");
    if (p->timing) return fail(p, SIGW_E_STATE, "disable timing before capturing a graph");
    if (n_sel < 1 || !slots) return fail(p, SIGW_E_INVALID, "need at least one slot");
    if (sigw_status s = check_targets(p, n_k, kt, lo, hi)) return s;
    if (n_k < 1) return fail(p, SIGW_E_INVALID, "need at least one target");
    if (long(n_sel) * n_k > kMaxTargets) return fail(p, SIGW_E_INVALID, "n_sel * n_k exceeds 4096");
    for (int i = 0; i < n_sel; ++i)
        if (slots[i] < 0 || slots[i] >= p->d.n_slots) return fail(p, SIGW_E_INVALID, "slot out of range");
    std::unique_ptr<sigw_graph> gr(new (std::nothrow) sigw_graph());
    if (!gr) return SIGW_E_NOMEM;
    gr->p = p;
    gr->grid_gen = p->grid_gen;
    gr->n_sel = n_sel;
    gr->n_k = n_k;
    gr->kt.assign(kt, kt + n_k);
    const size_t cnt = size_t(n_sel) * n_k;
    if (hipMalloc((void**)&gr->d_slots, size_t(n_sel) * 4) != hipSuccess ||
        hipMalloc((void**)&gr->d_sums, cnt * 8) != hipSuccess || hipMalloc((void**)&gr->d_cnts, cnt * 8) != hipSuccess ||
        hipHostMalloc((void**)&gr->h_sums, cnt * 8) != hipSuccess ||
        hipHostMalloc((void**)&gr->h_cnts, cnt * 8) != hipSuccess) {
        (void)hipGetLastError();
        sigw_graph_destroy(gr.release());
        return fail(p, SIGW_E_NOMEM, "graph buffers");
    }
    // the slot list is part of the graph's inputs, staged before capture
    if (hipMemcpy(gr->d_slots, slots, size_t(n_sel) * 4, hipMemcpyHostToDevice) != hipSuccess) {
        sigw_graph_destroy(gr.release());
        return fail(p, SIGW_E_DEVICE, "graph slot list upload");
    }
    if (hipStreamSynchronize(p->stream) != hipSuccess) {
        sigw_graph_destroy(gr.release());
        return fail(p, SIGW_E_DEVICE, "hipStreamSynchronize before capture");
    }
    if (hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        sigw_graph_destroy(gr.release());
        return fail(p, SIGW_E_DEVICE, "hipStreamBeginCapture (a graph needs a non-null plan stream)");
    }
    sigw_status s =
        enqueue_spectrum(p, gr->d_slots, n_sel, n_k, kt, lo, hi, gr->d_sums, gr->d_cnts, gr->valid, false);
    if (s == SIGW_OK) {
        if (hipMemcpyAsync(gr->h_sums, gr->d_sums, cnt * 8, hipMemcpyDeviceToHost, p->stream) != hipSuccess ||
            hipMemcpyAsync(gr->h_cnts, gr->d_cnts, cnt * 8, hipMemcpyDeviceToHost, p->stream) != hipSuccess)
            s = fail(p, SIGW_E_DEVICE, "result copies during capture");
    }
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(p->stream, &g);
    gr->g = g;
    if (s != SIGW_OK) {
        sigw_graph_destroy(gr.release());
        return s;
    }
    if (ec != hipSuccess || !g) {
        sigw_graph_destroy(gr.release());
        return fail(p, SIGW_E_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(ec));
    }
    if (hipGraphInstantiate(&gr->ge, gr->g, nullptr, nullptr, 0) != hipSuccess) {
        sigw_graph_destroy(gr.release());
        return fail(p, SIGW_E_DEVICE, "hipGraphInstantiate");
    }
    *out = gr.release();
    return SIGW_OK;
}

sigw_status sigw_graph_launch(sigw_graph_t gr) {
    if (!gr) return SIGW_E_INVALID;
    sigw_plan* p = gr->p;
    if (gr->grid_gen != p->grid_gen)
        return fail(p, SIGW_E_STATE, "the plan's u grid changed after this graph was captured: create it again");
    HIP_TRY(p, hipGraphLaunch(gr->ge, p->stream));
    gr->launched = true;
    return SIGW_OK;
}

sigw_status sigw_graph_results(sigw_graph_t gr, double* omega, int64_t* nmodes) {
    if (!gr) return SIGW_E_INVALID;
    sigw_plan* p = gr->p;
    if (!gr->launched) return fail(p, SIGW_E_STATE, "graph not launched");
    HIP_TRY(p, hipStreamSynchronize(p->stream));
    for (int i = 0; i < gr->n_sel; ++i)
        to_omega(p, gr->n_k, gr->kt.data(), gr->h_sums + size_t(i) * gr->n_k, gr->h_cnts + size_t(i) * gr->n_k,
                 gr->valid.data(), omega ? omega + size_t(i) * gr->n_k : nullptr,
                 nmodes ? nmodes + size_t(i) * gr->n_k : nullptr);
    return SIGW_OK;
}

sigw_status sigw_autotune(sigw_plan_t p, int32_t flags) {
    if (!p) return SIGW_E_INVALID;
    if (flags & ~int32_t(SIGW_TUNE_FORCE)) return fail(p, SIGW_E_INVALID, "unknown autotune flags");
    if (p->pending) return fail(p, SIGW_E_STATE, "an asynchronous spectrum is still in flight");
    HIP_TRY(p, hipStreamSynchronize(p->stream));
    return tune_xprod(p, flags);
}

sigw_status sigw_plan_schedule(sigw_plan_t p, int32_t* index, int32_t* count, char* text, size_t text_len) {
    if (!p) return SIGW_E_INVALID;
    if (index) *index = p->eng->xprod_schedule();
    if (count) *count = p->eng->xprod_schedules();
    if (text && text_len > 0) {
        const size_t n = std::min(text_len - 1, p->schedule.size());
        std::memcpy(text, p->schedule.data(), n);
        text[n] = '\0';
    }
    return SIGW_OK;
}

sigw_status sigw_plan_set_schedule(sigw_plan_t p, int32_t index) {
    if (!p) return SIGW_E_INVALID;
    if (index < 0 || index >= p->eng->xprod_schedules())
        return fail(p, SIGW_E_INVALID, "schedule index out of range");
    if (p->pending) return fail(p, SIGW_E_STATE, "an asynchronous spectrum is still in flight");
    HIP_TRY(p, hipStreamSynchronize(p->stream));
    p->eng->set_xprod_schedule(index);
    p->schedule = schedule_name(p->eng.get(), index);
    return SIGW_OK;
}

sigw_status sigw_synchronize(sigw_plan_t p) {
    if (!p) return SIGW_E_INVALID;
    HIP_TRY(p, hipStreamSynchronize(p->stream));
    return SIGW_OK;
}

sigw_status sigw_set_timing(sigw_plan_t p, int32_t enabled) {
    if (!p) return SIGW_E_INVALID;
    if (p->pending) return fail(p, SIGW_E_STATE, "an asynchronous spectrum is still in flight");
    p->timing = enabled != 0;
    for (int i = 0; i < kNumTimed; ++i) {
        p->t_sum[i] = 0;
        p->t_cnt[i] = 0;
    }
    p->ev_marks.clear();
    p->ev_used = 0;
    return SIGW_OK;
}

sigw_status sigw_kernel_time(sigw_plan_t p, const char* name, double* avg_ms, int64_t* launches) {
    if (!p || !name) return SIGW_E_INVALID;
    for (int i = 0; i < kNumTimed; ++i) {
        if (std::strcmp(name, kTimedNames[i]) == 0) {
            if (avg_ms) *avg_ms = p->t_cnt[i] ? p->t_sum[i] / double(p->t_cnt[i]) : 0.0;
            if (launches) *launches = p->t_cnt[i];
            return SIGW_OK;
        }
    }
    return fail(p, SIGW_E_INVALID, "unknown kernel name");
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free spectrum (sigw_spectrum_noalloc): for callers that cannot
// allocate device memory.  Every device buffer the call needs (twiddles,
// kernel tables, lookup tables, the per-target workspace, shell partials and
// sums) is carved out of one static array per device, `scratch`; the host
// code never names the array itself, only the device address that
// hipGetSymbolAddress returns for the current device.
// ---------------------------------------------------------------------------
namespace {
constexpr size_t kNoAllocBytes = size_t(64) << 20;   // SIGW_NOALLOC_BYTES in the header
constexpr int kNoAllocMaxN = 64;
}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

std::mutex g_scratch_mu;
std::map<int, char*> g_scratch_ptr;        // device ordinal -> its copy of `scratch`
thread_local std::string g_noalloc_err;    // text of the last failed no-alloc call

// Device address of the current device's copy of `scratch`, looked up once
// per device (with that device current) and kept.
hipError_t scratch_address(int dev, char** out) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it != g_scratch_ptr.end()) {
        *out = it->second;
        return hipSuccess;
    }
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = static_cast<char*>(ptr);
    *out = static_cast<char*>(ptr);
    return hipSuccess;
}

// Consecutive 256-byte aligned pieces of the scratch array; with base ==
// nullptr it only adds up the size of a layout.
struct Carve {
    char* base;
    size_t used = 0;
    void* take(size_t bytes) {
        const size_t o = (used + 255) & ~size_t(255);
        used = o + bytes;
        return base ? base + o : nullptr;
    }
};

// Lay out every device buffer of one allocation-free spectrum of desc d with
// `chunk` terms per x pass and `stage` staged terms, n_k targets; fills the
// plan's device pointers when base is set.  Returns the bytes used.
size_t noalloc_layout(sigw_plan* p, char* base, int n_k) {
    const sigw_plan_desc& d = p->d;
    const Sizes& z = p->z;
    Carve c{base};
    p->tw = c.take(size_t(d.N) * z.cb);
    p->edges = static_cast<double*>(c.take(size_t(d.n_modes + 1) * 8));
    for (int m = 0; m < 2; ++m) {
        p->phi_tab[m] = c.take(size_t(d.n_modes) * d.n_alpha * z.rb);
        p->sigma_tab[m] = c.take(size_t(d.n_alpha) * z.rb);
    }
    p->lut_u = static_cast<int16_t*>(c.take(size_t(z.n2max + 1) * 2));
    p->lut_shell = static_cast<uint8_t*>(c.take(size_t(z.n2max + 1)));
    p->T = c.take(size_t(3) * z.chunk * z.FS * z.cb);
    p->Sst = c.take(size_t(2) * z.stage * z.FS * z.cb);
    p->Q = c.take(size_t(12) * z.FS * z.cb);
    const size_t zb = size_t(z.H) * d.N;
    p->part_sum = static_cast<double*>(c.take(zb * 8));
    p->part_cnt = static_cast<unsigned long long*>(c.take(zb * 8));
    p->sums = static_cast<double*>(c.take(size_t(std::max(n_k, 1)) * 8));
    p->cnts = static_cast<unsigned long long*>(c.take(size_t(std::max(n_k, 1)) * 8));
    p->d_sel = static_cast<int*>(c.take(4));     // the slot list {0}; also the member list
    p->d_iota = p->d_sel;
    long fs_c = 0;
    for (size_t i = 0; i < p->coarse.size(); ++i) {
        const int m = kGridSizes[i];
        p->coarse[i].tw = c.take(size_t(m) * z.cb);
        fs_c = long(m / 2 + 1) * m * m;
    }
    p->phi_c = fs_c ? c.take(size_t(fs_c) * z.cb) : nullptr;
    return c.used;
}

const char* g_noalloc_err_text() { return g_noalloc_err.c_str(); }

sigw_status noalloc_fail(sigw_status s, const std::string& msg) {
    g_noalloc_err = msg;
    return s;
}

}  // namespace

extern "C" sigw_status sigw_spectrum_noalloc(const sigw_plan_desc* d, const void* phi_hat_dev, int32_t n_k,
                                             const double* kt, const double* lo, const double* hi,
                                             double* omega, int64_t* nmodes, void* hip_stream) {
    g_noalloc_err.clear();
    if (const char* why = validate(d)) return noalloc_fail(SIGW_E_INVALID, why);
    if (d->N > kNoAllocMaxN) return noalloc_fail(SIGW_E_INVALID, "the allocation-free spectrum takes N <= 64");
    if (!phi_hat_dev) return noalloc_fail(SIGW_E_INVALID, "NULL Phi_hat");
    sigw_plan P;                     // host-side state only; its device pointers point into scratch
    P.d = *d;
    P.d.n_slots = 1;
    P.d.batch = 1;
    P.stream = static_cast<hipStream_t>(hip_stream);
    if (sigw_status s = check_targets(&P, n_k, kt, lo, hi)) return noalloc_fail(s, P.err);
    try {
        P.lattice_n2 = lattice_n2_table(d->N);
        const std::shared_ptr<const Decomposition> dec = decomposition_of(*d);
        P.edges_h = dec->edges;
        for (int m = 0; m < 2; ++m) P.tab_h[m] = dec->tab[m];
        for (int m : kGridSizes)
            if (m < d->N) P.coarse.emplace_back().N = m;
    } catch (const std::bad_alloc&) {
        return noalloc_fail(SIGW_E_NOMEM, "host memory");
    }
    // Terms per x pass and staged terms: the caller's, or (0) the largest
    // count up to n_alpha whose layout fits the array.
    auto fits = [&](int chunk, int stage) {
        P.d.alpha_chunk = chunk;
        P.d.scratch_terms = stage;
        P.z = sizes_of(P.d);
        return noalloc_layout(&P, nullptr, n_k) <= kNoAllocBytes;
    };
    const int want_chunk = d->alpha_chunk, want_stage = d->scratch_terms;
    int chunk = want_chunk ? want_chunk : d->n_alpha;
    while (chunk > 1 && !fits(chunk, want_stage ? std::min(want_stage, chunk) : 1) && !want_chunk) --chunk;
    int stage = want_stage ? std::min(want_stage, chunk) : chunk;
    while (stage > 1 && !fits(chunk, stage) && !want_stage) --stage;
    if (!fits(chunk, stage))
        return noalloc_fail(SIGW_E_INVALID, "this lattice, precision and term counts need more than the " +
                                                std::to_string(kNoAllocBytes >> 20) +
                                                " MiB of the allocation-free buffer (lower alpha_chunk or scratch_terms)");
    // only now touch the device: the address of its copy of the array
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return noalloc_fail(SIGW_E_DEVICE, "hipGetDevice failed");
    char* base = nullptr;
    if (hipError_t e = scratch_address(dev, &base); e != hipSuccess)
        return noalloc_fail(SIGW_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    noalloc_layout(&P, base, n_k);
    P.phi_hat = const_cast<void*>(phi_hat_dev);
    P.has_field.assign(1, 1);
    // tables in the path precision, twiddles, the slot list {0}
    const Sizes& z = P.z;
    std::vector<char> twh(size_t(d->N) * z.cb), phih[2], sigh[2];
    sigw::host_twiddles(d->prec, d->N, twh.data());
    std::vector<std::vector<char>> twc(P.coarse.size());
    for (size_t i = 0; i < P.coarse.size(); ++i) {
        twc[i].resize(size_t(P.coarse[i].N) * z.cb);
        sigw::host_twiddles(d->prec, P.coarse[i].N, twc[i].data());
    }
    for (int m = 0; m < 2; ++m) {
        const Table& t = P.tab_h[m];
        phih[m].resize(t.phi.size() * z.rb);
        sigh[m].resize(t.sigma.size() * z.rb);
        for (size_t i = 0; i < t.phi.size(); ++i) {
            if (d->prec == SIGW_F64) reinterpret_cast<double*>(phih[m].data())[i] = t.phi[i];
            else reinterpret_cast<float*>(phih[m].data())[i] = float(t.phi[i]);
        }
        for (size_t i = 0; i < t.sigma.size(); ++i) {
            if (d->prec == SIGW_F64) reinterpret_cast<double*>(sigh[m].data())[i] = t.sigma[i];
            else reinterpret_cast<float*>(sigh[m].data())[i] = float(t.sigma[i]);
        }
    }
    const int zero = 0;
    hipStream_t s = P.stream;
    bool ok = hipMemcpyAsync(P.tw, twh.data(), twh.size(), hipMemcpyHostToDevice, s) == hipSuccess &&
              hipMemcpyAsync(P.edges, P.edges_h.data(), P.edges_h.size() * 8, hipMemcpyHostToDevice, s) == hipSuccess &&
              hipMemcpyAsync(P.d_sel, &zero, 4, hipMemcpyHostToDevice, s) == hipSuccess;
    for (int m = 0; m < 2 && ok; ++m)
        ok = hipMemcpyAsync(P.phi_tab[m], phih[m].data(), phih[m].size(), hipMemcpyHostToDevice, s) == hipSuccess &&
             hipMemcpyAsync(P.sigma_tab[m], sigh[m].data(), sigh[m].size(), hipMemcpyHostToDevice, s) == hipSuccess;
    for (size_t i = 0; i < P.coarse.size() && ok; ++i)
        ok = hipMemcpyAsync(P.coarse[i].tw, twc[i].data(), twc[i].size(), hipMemcpyHostToDevice, s) == hipSuccess;
    if (!ok) {
        (void)hipStreamSynchronize(s);
        return noalloc_fail(SIGW_E_DEVICE, "table upload failed");
    }
    P.eng.reset(sigw::make_engine(d->prec, d->N, P.tw));
    for (auto& c : P.coarse) c.eng.reset(sigw::make_engine(d->prec, c.N, c.tw));
    bool made = bool(P.eng);
    for (auto& c : P.coarse) made = made && bool(c.eng);
    if (!made) {
        (void)hipStreamSynchronize(s);
        return noalloc_fail(SIGW_E_UNSUPPORTED, "no compiled schedule for this size");
    }
    std::vector<int> valid;
    sigw_status st = enqueue_spectrum(&P, P.d_sel, 1, n_k, kt, lo, hi, P.sums, P.cnts, valid, false);
    std::vector<double> hs(size_t(std::max(n_k, 1)), 0.0);
    std::vector<unsigned long long> hc(size_t(std::max(n_k, 1)), 0ull);
    if (st == SIGW_OK && n_k > 0 &&
        (hipMemcpyAsync(hs.data(), P.sums, size_t(n_k) * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
         hipMemcpyAsync(hc.data(), P.cnts, size_t(n_k) * 8, hipMemcpyDeviceToHost, s) != hipSuccess))
        st = fail(&P, SIGW_E_DEVICE, "result copies failed");
    // the host tables above must outlive their copies: wait for the stream in every case
    const hipError_t es = hipStreamSynchronize(s);
    if (st != SIGW_OK) return noalloc_fail(st, P.err);
    if (es != hipSuccess) return noalloc_fail(SIGW_E_DEVICE, std::string("hipStreamSynchronize: ") + hipGetErrorString(es));
    to_omega(&P, n_k, kt, hs.data(), hc.data(), valid.data(), omega, nmodes);
    return SIGW_OK;
}
