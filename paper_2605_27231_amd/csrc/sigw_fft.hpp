// Device-side FFT building blocks for gfx950: complex arithmetic, radix-2/3/4/8
// butterflies, register DFTs of composite size with compile-time twiddles,
// and the two-phase line transform (register DFT, LDS transpose, register
// DFT) that every pass of the pipeline is built from.  Sign convention:
// out[p] = sum_m a[m] exp(sign 2 pi i m p / r); the forward transform uses
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

// ----------------------------------------------------------------------------
// Register DFTs of composite size (four-step inside one thread).  Their
// twiddles are exp(sign 2 pi i m / R) with R dividing 96 and m fixed once the
// loops are unrolled, so they are immediate constants, and the trivial ones
// (1, -1, +-i) cost no multiplication.
// ----------------------------------------------------------------------------
// cos(2 pi m / 96) for m = 0..24, correctly rounded
__device__ constexpr double kCos96[25] = {
    1.0, 0.99785892323860350673807, 0.991444861373810411144558,
    0.980785280403230449126182, 0.965925826289068286749743, 0.946930129495105664255804,
    0.923879532511286756128183, 0.896872741532688303894104, 0.866025403784438646763723,
    0.831469612302545237078788, 0.793353340291235164579777, 0.751839807478977396407519,
    0.707106781186547524400844, 0.659345815100068868425125, 0.608761429008720639416098,
    0.555570233019602224742831, 0.5, 0.442288690219001281995239,
    0.38268343236508977172846, 0.321439465303161580701058, 0.258819045102520762348899,
    0.195090322016128267848285, 0.130526192220051591548406, 0.065403129230143066815316,
    0.0,
};

__device__ constexpr double cos96(int e) {
    e = ((e % 96) + 96) % 96;
    return e <= 24 ? kCos96[e] : e <= 48 ? -kCos96[48 - e] : e <= 72 ? -kCos96[e - 48] : kCos96[96 - e];
}

// a * exp(sign 2 pi i m / R); m is a constant after unrolling, so the
// branches fold away
template <int SIGN, int R, typename C> __device__ __forceinline__ C ctw_mul(C a, int m) {
    static_assert(96 % R == 0, "register DFT twiddles are multiples of 2 pi / 96");
    using T = decltype(C::x);
    const int e = (m % R) * (96 / R);
    if (e == 0) return a;
    if (e == 48) return cmk<C>(-a.x, -a.y);
    if (e == 24) return mul_si<SIGN>(a);
    if (e == 72) return mul_si<-SIGN>(a);
    const T c = T(cos96(e)), s = T(SIGN) * T(cos96(e - 24));
    return cmk<C>(a.x * c - a.y * s, a.x * s + a.y * c);
}

template <int R> struct RegSplit;                 // R = F * G, F a base radix
template <> struct RegSplit<12> { static constexpr int F = 4, G = 3; };
template <> struct RegSplit<16> { static constexpr int F = 4, G = 4; };
template <> struct RegSplit<24> { static constexpr int F = 8, G = 3; };
template <> struct RegSplit<32> { static constexpr int F = 8, G = 4; };

// Inter-phase twiddle exp(sign 2 pi i e / N) from the table tw[t] =
// exp(-2 pi i t / N) (in global memory or an LDS copy).
template <int SIGN, int N, typename C>
__device__ __forceinline__ C tw_at(const C* tw, int e) {
    C w = tw[e];
    if (SIGN > 0) w.y = -w.y;
    return w;
}

template <int R, int SIGN, typename C>
__device__ __forceinline__ void reg_dft(C* a) {
    if constexpr (R == 1) {
    } else if constexpr (R == 2 || R == 3 || R == 4 || R == 8) {
        dft<R, SIGN>(a);
    } else {
        constexpr int F = RegSplit<R>::F;
        constexpr int G = RegSplit<R>::G;
        static_assert(F * G == R, "bad split");
        C tmp[R];
        // x index n = g + G f; out index k = kf + F kg
#pragma unroll
        for (int g = 0; g < G; ++g) {
            C v[F];
#pragma unroll
            for (int f = 0; f < F; ++f) v[f] = a[g + G * f];
            dft<F, SIGN>(v);
#pragma unroll
            for (int kf = 0; kf < F; ++kf) tmp[g * F + kf] = ctw_mul<SIGN, R>(v[kf], g * kf);
        }
#pragma unroll
        for (int kf = 0; kf < F; ++kf) {
            C w[G];
#pragma unroll
            for (int g = 0; g < G; ++g) w[g] = tmp[g * F + kf];
            reg_dft<G, SIGN>(w);
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
// lds must hold TPLayout<N, NL, LINE_FAST>::size complex values (NL * N
// plus padding).  The phases contain no barrier: the caller synchronises
// between phase 1 and phase 2 and before the buffer is reused.
// ----------------------------------------------------------------------------
// R1_ = 0 takes the size's default factorisation (TwoPhase), another value
// a different first radix for the same N.
template <int N, int NL, bool LINE_FAST, int R1_ = 0> struct TPLayout {
    static constexpr int R1 = R1_ ? R1_ : TwoPhase<N>::R1;
    static_assert(N % R1 == 0, "the first radix divides N");
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

// The inter-phase twiddles of phase 1 as an R1 x R2 matrix in LDS:
// twm[k1 R2 + t] = exp(-2 pi i t k1 / N).  Lanes of one phase-1 pass hold
// consecutive t, so they read consecutive entries (no bank conflicts, unlike
// the strided entries t k1 of the plain table).
template <typename C, int N, int R1, int NT>
__device__ __forceinline__ void stage_twiddle_matrix(C* twm, const C* __restrict__ tw, int tid) {
    constexpr int R2 = N / R1;
    for (int i = tid; i < N; i += NT) twm[i] = tw[((i % R2) * (i / R2)) % N];
}

// Phase 1 of one item whose inputs are already in registers: a[m] holds
// element t + R2 m of line `line`; a is overwritten.  The inter-phase
// twiddles tw[t k1] depend on the lane: with tw a copy of the table in LDS
// they stay off the vector memory path.  TWM: tw is the twiddle matrix of
// stage_twiddle_matrix instead of the plain table.
template <typename C, int N, int SIGN, int NL, bool LINE_FAST, int R1_ = 0, bool TWM = false>
__device__ __forceinline__ void tp_phase1_item(C* a, int line, int t, C* lds, const C* tw) {
    using Lay = TPLayout<N, NL, LINE_FAST, R1_>;
    constexpr int R1 = Lay::R1, R2 = Lay::R2;
    reg_dft<R1, SIGN>(a);
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) {
        C v = a[k1];
        if (k1 > 0) v = cmul(v, TWM ? tw_at<SIGN, N>(tw, k1 * R2 + t) : tw_at<SIGN, N>(tw, t * k1));
        lds[Lay::at(line, k1, t)] = v;
    }
}

// Phase 1 over all NL lines, items spread over NT threads; ld(line, n)
// returns element n of a line.
template <typename C, int N, int SIGN, int NL, int NT, bool LINE_FAST, bool TWM = false, class LD>
__device__ __forceinline__ void tp_phase1(LD&& ld, C* lds, const C* tw, int tid) {
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
            tp_phase1_item<C, N, SIGN, NL, LINE_FAST, 0, TWM>(a, line, t, lds, tw);
        }
    }
}

// As tp_phase1, with ld(line, t, m) returning element t + R2 m of a line;
// m is a constant once the loop is unrolled, so ld can branch on it freely.
template <typename C, int N, int SIGN, int NL, int NT, bool LINE_FAST, int R1_ = 0, class LD>
__device__ __forceinline__ void tp_phase1_tm(LD&& ld, C* lds, const C* tw, int tid) {
    using Lay = TPLayout<N, NL, LINE_FAST, R1_>;
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
            for (int m = 0; m < R1; ++m) a[m] = ld(line, t, m);
            tp_phase1_item<C, N, SIGN, NL, LINE_FAST, R1_>(a, line, t, lds, tw);
        }
    }
}

// Copy of the N-entry twiddle table into LDS, for the lane-dependent twiddles
// of phase 1 (the caller synchronises before use).
template <typename C, int N, int NT>
__device__ __forceinline__ void stage_twiddles(C* twl, const C* __restrict__ tw, int tid) {
#pragma unroll
    for (int i = tid; i < N; i += NT) twl[i] = tw[i];
}

template <typename C, int N, int SIGN, int NL, int NT, bool LINE_FAST, int R1_ = 0, class ST>
__device__ __forceinline__ void tp_phase2(ST&& st, const C* lds, int tid) {
    using Lay = TPLayout<N, NL, LINE_FAST, R1_>;
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
            reg_dft<R2, SIGN>(b);
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
    __device__ __forceinline__ void run(const C* lds, int tid) {
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int w = tid + i * NT;
            if ((ITEMS % NT == 0) || w < ITEMS) {
                const int line = LINE_FAST ? w % NL : w / R1;
                const int k1 = LINE_FAST ? w / NL : w % R1;
#pragma unroll
                for (int t = 0; t < R2; ++t) v[i][t] = lds[Lay::at(line, k1, t)];
                reg_dft<R2, SIGN>(v[i]);
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
