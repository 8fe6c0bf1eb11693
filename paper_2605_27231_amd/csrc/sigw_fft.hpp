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

}  // namespace sigw
