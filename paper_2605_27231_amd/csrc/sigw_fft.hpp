// Device-side FFT building blocks for gfx950: complex arithmetic, radix-2/3/4/8
// butterflies and a Stockham autosort pass sequence that runs NL independent
// lines of length N held in LDS, with NT threads of the workgroup.
//
// Stockham step (radix r, L = product of the radices already applied):
//   for j in [0, N/r):  k = j mod L
//     a_m = x[j + m N/r] * w^(m k),  w = exp(sign 2 pi i / (L r)),  m = 0..r-1
//     b_p = sum_m a_m exp(sign 2 pi i m p / r)
//     y[(j - k) r + k + p L] = b_p
// After all steps the output is in natural order.  The forward transform uses
// sign = -1, the inverse sign = +1 (unnormalised).
#pragma once

#include <hip/hip_runtime.h>

namespace sigw {

template <typename R> struct CplxOf;
template <> struct CplxOf<float> { using T = float2; };
template <> struct CplxOf<double> { using T = double2; };

template <typename C> __device__ __forceinline__ C cmk(decltype(C::x) a, decltype(C::x) b) {
    C r;
    r.x = a;
    r.y = b;
    return r;
}
template <typename C> __device__ __forceinline__ C cadd(C a, C b) { return cmk<C>(a.x + b.x, a.y + b.y); }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { return cmk<C>(a.x - b.x, a.y - b.y); }
template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
    return cmk<C>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename C> __device__ __forceinline__ C cconj(C a) { return cmk<C>(a.x, -a.y); }
template <typename C, typename S> __device__ __forceinline__ C cscale(C a, S s) {
    return cmk<C>(a.x * s, a.y * s);
}
// a * (sign * i)
template <int SIGN, typename C> __device__ __forceinline__ C mul_si(C a) {
    return SIGN > 0 ? cmk<C>(-a.y, a.x) : cmk<C>(a.y, -a.x);
}

// ---- butterflies: in place, out[p] = sum_m a[m] exp(sign 2 pi i m p / r) ----
template <int SIGN, typename C> __device__ __forceinline__ void dft2(C* a) {
    C t = a[0];
    a[0] = cadd(t, a[1]);
    a[1] = csub(t, a[1]);
}

template <int SIGN, typename C> __device__ __forceinline__ void dft3(C* a) {
    using R = decltype(C::x);
    const R h = R(0.86602540378443864676);   // sqrt(3)/2
    C s = cadd(a[1], a[2]);
    C d = csub(a[1], a[2]);
    C m = cmk<C>(a[0].x - R(0.5) * s.x, a[0].y - R(0.5) * s.y);
    C t = mul_si<SIGN>(cscale(d, h));
    a[0] = cadd(a[0], s);
    a[1] = cadd(m, t);
    a[2] = csub(m, t);
}

template <int SIGN, typename C> __device__ __forceinline__ void dft4(C* a) {
    C t0 = cadd(a[0], a[2]);
    C t1 = csub(a[0], a[2]);
    C t2 = cadd(a[1], a[3]);
    C t3 = mul_si<SIGN>(csub(a[1], a[3]));
    a[0] = cadd(t0, t2);
    a[2] = csub(t0, t2);
    a[1] = cadd(t1, t3);
    a[3] = csub(t1, t3);
}

template <int SIGN, typename C> __device__ __forceinline__ void dft8(C* a) {
    using R = decltype(C::x);
    const R r2 = R(0.70710678118654752440);
    C e[4] = {a[0], a[2], a[4], a[6]};
    C o[4] = {a[1], a[3], a[5], a[7]};
    dft4<SIGN>(e);
    dft4<SIGN>(o);
    // w^1 = (1 + sign i)/sqrt2, w^2 = sign i, w^3 = (-1 + sign i)/sqrt2
    C o1 = cscale(cadd(o[1], mul_si<SIGN>(o[1])), r2);
    C o2 = mul_si<SIGN>(o[2]);
    C o3 = cscale(csub(mul_si<SIGN>(o[3]), o[3]), r2);
    a[0] = cadd(e[0], o[0]);
    a[4] = csub(e[0], o[0]);
    a[1] = cadd(e[1], o1);
    a[5] = csub(e[1], o1);
    a[2] = cadd(e[2], o2);
    a[6] = csub(e[2], o2);
    a[3] = cadd(e[3], o3);
    a[7] = csub(e[3], o3);
}

template <int R_, int SIGN, typename C> __device__ __forceinline__ void dft(C* a) {
    if constexpr (R_ == 2) dft2<SIGN>(a);
    else if constexpr (R_ == 3) dft3<SIGN>(a);
    else if constexpr (R_ == 4) dft4<SIGN>(a);
    else if constexpr (R_ == 8) dft8<SIGN>(a);
    else static_assert(R_ == 2, "unsupported radix");
}

// ---- radix schedules (product = N) ----
template <int N> struct Radices;
template <> struct Radices<8> { static constexpr int n = 1; static constexpr int r[1] = {8}; };
template <> struct Radices<16> { static constexpr int n = 2; static constexpr int r[2] = {4, 4}; };
template <> struct Radices<32> { static constexpr int n = 2; static constexpr int r[2] = {8, 4}; };
template <> struct Radices<64> { static constexpr int n = 2; static constexpr int r[2] = {8, 8}; };
template <> struct Radices<128> { static constexpr int n = 3; static constexpr int r[3] = {8, 4, 4}; };
template <> struct Radices<256> { static constexpr int n = 3; static constexpr int r[3] = {8, 8, 4}; };
template <> struct Radices<384> { static constexpr int n = 4; static constexpr int r[4] = {8, 8, 2, 3}; };
template <> struct Radices<512> { static constexpr int n = 3; static constexpr int r[3] = {8, 8, 8}; };

// One Stockham step over NL lines; line l, element e lives at buf[l*LS + e*ES].
// tw[t] = exp(-2 pi i t / N), t = 0..N-1.
template <typename C, int N, int RD, int L, int NL, int NT, int SIGN, int LS, int ES>
__device__ __forceinline__ void stockham_step(C* buf, const C* __restrict__ tw, int tid) {
    constexpr int M = N / RD;
    constexpr int NB = NL * M;
    constexpr int PER = (NB + NT - 1) / NT;
    C v[PER][RD];
#pragma unroll
    for (int p = 0; p < PER; ++p) {
        const int b = tid + p * NT;
        if ((NB % NT == 0) || b < NB) {
            const int line = b / M;
            const int j = b - line * M;
#pragma unroll
            for (int m = 0; m < RD; ++m) v[p][m] = buf[line * LS + (j + m * M) * ES];
        }
    }
    __syncthreads();
#pragma unroll
    for (int p = 0; p < PER; ++p) {
        const int b = tid + p * NT;
        if ((NB % NT == 0) || b < NB) {
            const int line = b / M;
            const int j = b - line * M;
            const int k = j % L;
            if constexpr (L > 1) {
#pragma unroll
                for (int m = 1; m < RD; ++m) {
                    C w = tw[(m * k) * (N / (L * RD))];
                    if (SIGN > 0) w.y = -w.y;
                    v[p][m] = cmul(v[p][m], w);
                }
            }
            dft<RD, SIGN>(v[p]);
            const int base = (j - k) * RD + k;
#pragma unroll
            for (int m = 0; m < RD; ++m) buf[line * LS + (base + m * L) * ES] = v[p][m];
        }
    }
    __syncthreads();
}

template <typename C, int N, int NL, int NT, int SIGN, int LS, int ES, int S, int L>
__device__ __forceinline__ void stockham_from(C* buf, const C* __restrict__ tw, int tid) {
    if constexpr (S < Radices<N>::n) {
        constexpr int RD = Radices<N>::r[S];
        stockham_step<C, N, RD, L, NL, NT, SIGN, LS, ES>(buf, tw, tid);
        stockham_from<C, N, NL, NT, SIGN, LS, ES, S + 1, L * RD>(buf, tw, tid);
    }
}

// Full length-N transform of NL lines in LDS.  The caller has synchronised
// after filling buf; on return every thread may read the result.
template <typename C, int N, int NL, int NT, int SIGN, int LS, int ES>
__device__ __forceinline__ void lds_fft(C* buf, const C* __restrict__ tw, int tid) {
    stockham_from<C, N, NL, NT, SIGN, LS, ES, 0, 1>(buf, tw, tid);
}


// ----------------------------------------------------------------------------
// Register DFTs of composite size (four-step inside one thread).
// Twiddles come from the length-N table tw[t] = exp(-2 pi i t / N) at
// compile-time offsets, so they are uniform (scalar) loads.
// ----------------------------------------------------------------------------
template <int R> struct RegSplit;                 // R = F * G, F a base radix
template <> struct RegSplit<12> { static constexpr int F = 4, G = 3; };
template <> struct RegSplit<16> { static constexpr int F = 4, G = 4; };
template <> struct RegSplit<24> { static constexpr int F = 8, G = 3; };
template <> struct RegSplit<32> { static constexpr int F = 8, G = 4; };

template <int SIGN, int N, typename C>
__device__ __forceinline__ C tw_at(const C* __restrict__ tw, int e) {
    C w = tw[e];
    if (SIGN > 0) w.y = -w.y;
    return w;
}

template <int R, int SIGN, int N, typename C>
__device__ __forceinline__ void reg_dft(C* a, const C* __restrict__ tw) {
    if constexpr (R == 1) {
    } else if constexpr (R == 2 || R == 3 || R == 4 || R == 8) {
        dft<R, SIGN>(a);
    } else {
        constexpr int F = RegSplit<R>::F;
        constexpr int G = RegSplit<R>::G;
        static_assert(F * G == R, "bad split");
        static_assert(N % R == 0, "register DFT size must divide N");
        C tmp[R];
        // x index n = g + G f; out index k = kf + F kg
#pragma unroll
        for (int g = 0; g < G; ++g) {
            C v[F];
#pragma unroll
            for (int f = 0; f < F; ++f) v[f] = a[g + G * f];
            dft<F, SIGN>(v);
#pragma unroll
            for (int kf = 0; kf < F; ++kf) {
                if (g * kf == 0) tmp[g * F + kf] = v[kf];
                else tmp[g * F + kf] = cmul(v[kf], tw_at<SIGN, N>(tw, ((g * kf) % R) * (N / R)));
            }
        }
#pragma unroll
        for (int kf = 0; kf < F; ++kf) {
            C w[G];
#pragma unroll
            for (int g = 0; g < G; ++g) w[g] = tmp[g * F + kf];
            reg_dft<G, SIGN, N>(w, tw);
#pragma unroll
            for (int kg = 0; kg < G; ++kg) a[kf + F * kg] = w[kg];
        }
    }
}

// Factorisation N = R1 * R2 used by the two-phase line transform.
template <int N> struct TwoPhase;
template <> struct TwoPhase<8> { static constexpr int R1 = 2; };
template <> struct TwoPhase<16> { static constexpr int R1 = 4; };
template <> struct TwoPhase<32> { static constexpr int R1 = 4; };
template <> struct TwoPhase<64> { static constexpr int R1 = 8; };
template <> struct TwoPhase<128> { static constexpr int R1 = 8; };
template <> struct TwoPhase<256> { static constexpr int R1 = 16; };
template <> struct TwoPhase<384> { static constexpr int R1 = 16; };
template <> struct TwoPhase<512> { static constexpr int R1 = 16; };

// ----------------------------------------------------------------------------
// Two-phase transform of NL lines of length N = R1 R2 (four-step):
//   phase 1, item (line, t), t < R2:  a_k1 = W_N^{t k1} sum_m x[t + R2 m] W_R1^{m k1}
//   LDS transpose
//   phase 2, item (line, k1), k1 < R1: X[k1 + R1 k2] = sum_t a_k1(t) W_R2^{t k2}
// ld(line, n) supplies x; st(line, k, X) consumes the output.  LINE_FAST puts
// consecutive threads on consecutive lines (for tiles whose lines are
// interleaved in memory); otherwise consecutive threads walk along a line.
// lds must hold NL * N complex (plus NL * R1 for the !LINE_FAST padding).
// The routine starts and ends without a barrier of its own on the LDS
// buffer other than the one between the phases; the caller synchronises
// before lds is reused.
// ----------------------------------------------------------------------------
template <int N, int NL, bool LINE_FAST> struct TPLayout {
    static constexpr int R1 = TwoPhase<N>::R1;
    static constexpr int R2 = N / R1;
    // LINE_FAST rows of one k1 hold R2 * NL elements.  When NL is not a
    // multiple of 16, the 16 lanes the LDS serves together span two k1 rows;
    // pad each row so that the next one starts NL elements further along the
    // banks (row stride = NL mod 32 elements) and those lanes do not collide.
    static constexpr int PADK = (NL % 16 == 0) ? 0 : ((NL - (R2 * NL) % 32) % 32 + 32) % 32;
    static constexpr int RS = R2 * NL + PADK;
    static constexpr int size = LINE_FAST ? R1 * RS : NL * R1 * (R2 + 1);
    __device__ static __forceinline__ int at(int line, int k1, int t) {
        return LINE_FAST ? k1 * RS + t * NL + line : (line * R1 + k1) * (R2 + 1) + t;
    }
};

// Phase 1.  tw serves the register DFT's own twiddles (fixed indices, read
// through the scalar cache); twv serves the inter-phase twiddles
// tw[t k1], whose index depends on the lane: a copy of the table in LDS
// keeps those off the vector memory path.
template <typename C, int N, int SIGN, int NL, int NT, bool LINE_FAST, class LD>
__device__ __forceinline__ void tp_phase1(LD&& ld, C* lds, const C* __restrict__ tw, const C* twv, int tid) {
    using Lay = TPLayout<N, NL, LINE_FAST>;
    constexpr int R1 = Lay::R1, R2 = Lay::R2;
    constexpr int ITEMS = NL * R2;
#pragma unroll
    for (int w0 = 0; w0 < ITEMS; w0 += NT) {
        const int w = w0 + tid;
        if ((ITEMS % NT == 0) || w < ITEMS) {
            const int line = LINE_FAST ? w % NL : w / R2;
            const int t = LINE_FAST ? w / NL : w % R2;
            C a[R1];
#pragma unroll
            for (int m = 0; m < R1; ++m) a[m] = ld(line, t + R2 * m);
            reg_dft<R1, SIGN, N>(a, tw);
#pragma unroll
            for (int k1 = 0; k1 < R1; ++k1) {
                C v = a[k1];
                if (k1 > 0) v = cmul(v, tw_at<SIGN, N>(twv, t * k1));
                lds[Lay::at(line, k1, t)] = v;
            }
        }
    }
}

template <typename C, int N, int SIGN, int NL, int NT, bool LINE_FAST, class LD>
__device__ __forceinline__ void tp_phase1(LD&& ld, C* lds, const C* __restrict__ tw, int tid) {
    tp_phase1<C, N, SIGN, NL, NT, LINE_FAST>(ld, lds, tw, tw, tid);
}

// Copy of the N-entry twiddle table into LDS, for the lane-dependent twiddles
// of phase 1 (the caller synchronises before use).
template <typename C, int N, int NT>
__device__ __forceinline__ void stage_twiddles(C* twl, const C* __restrict__ tw, int tid) {
#pragma unroll
    for (int i = tid; i < N; i += NT) twl[i] = tw[i];
}

template <typename C, int N, int SIGN, int NL, int NT, bool LINE_FAST, class ST>
__device__ __forceinline__ void tp_phase2(ST&& st, const C* lds, const C* __restrict__ tw, int tid) {
    using Lay = TPLayout<N, NL, LINE_FAST>;
    constexpr int R1 = Lay::R1, R2 = Lay::R2;
    constexpr int ITEMS = NL * R1;
#pragma unroll
    for (int w0 = 0; w0 < ITEMS; w0 += NT) {
        const int w = w0 + tid;
        if ((ITEMS % NT == 0) || w < ITEMS) {
            const int line = LINE_FAST ? w % NL : w / R1;
            const int k1 = LINE_FAST ? w / NL : w % R1;
            C b[R2];
#pragma unroll
            for (int t = 0; t < R2; ++t) b[t] = lds[Lay::at(line, k1, t)];
            reg_dft<R2, SIGN, N>(b, tw);
#pragma unroll
            for (int k2 = 0; k2 < R2; ++k2) st(line, k1 + R1 * k2, b[k2]);
        }
    }
}

// Phase 2 into registers: out[i][k2] for the i-th item of this thread
// (item w = tid + i NT), so that the caller can synchronise before storing
// into the same LDS buffer.
template <typename C, int N, int SIGN, int NL, int NT, bool LINE_FAST>
struct TPRegs {
    using Lay = TPLayout<N, NL, LINE_FAST>;
    static constexpr int R1 = Lay::R1, R2 = Lay::R2;
    static constexpr int ITEMS = NL * R1;
    static constexpr int PER = (ITEMS + NT - 1) / NT;
    C v[PER][R2];
    __device__ __forceinline__ void run(const C* lds, const C* __restrict__ tw, int tid) {
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int w = tid + i * NT;
            if ((ITEMS % NT == 0) || w < ITEMS) {
                const int line = LINE_FAST ? w % NL : w / R1;
                const int k1 = LINE_FAST ? w / NL : w % R1;
#pragma unroll
                for (int t = 0; t < R2; ++t) v[i][t] = lds[Lay::at(line, k1, t)];
                reg_dft<R2, SIGN, N>(v[i], tw);
            }
        }
    }
    template <class ST> __device__ __forceinline__ void store(ST&& st, int tid) {
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int w = tid + i * NT;
            if ((ITEMS % NT == 0) || w < ITEMS) {
                const int line = LINE_FAST ? w % NL : w / R1;
                const int k1 = LINE_FAST ? w / NL : w % R1;
#pragma unroll
                for (int k2 = 0; k2 < R2; ++k2) st(line, k1 + R1 * k2, v[i][k2]);
            }
        }
    }
};

}  // namespace sigw
