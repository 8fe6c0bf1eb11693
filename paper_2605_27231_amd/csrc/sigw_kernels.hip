// HIP kernels of the Omega_GW lattice path for gfx950 (CDNA4, wave64).
//
// Data layouts (row-major, last index fastest):
//   real field    [x][y][z]                   N^3 reals
//   half spectrum [kx][ky][kz], kx = 0..N/2   (N/2+1) N^2 complex
// A 3D inverse transform runs z (complex, contiguous rows), then y (complex,
// strided), then x (the halved axis, complex-to-real); the forward transform
// runs the same passes in reverse order.  Every pass stages a tile through
// LDS so that global accesses are runs of at least 64-128 contiguous bytes.
//
// The hot loop for one target k fuses the Fourier weighting into the first
// inverse pass (gen_z), the products and the first forward pass into the last
// inverse pass (xprod), and the TT projection and FP64 shell sums into the
// last forward pass (zbin).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <type_traits>

#include "sigw_engine.hpp"
#include "sigw_fft.hpp"

namespace sigw {

// ----------------------------------------------------------------------------
// Tile shapes per (precision, N)
// ----------------------------------------------------------------------------
template <typename R, int N> struct Shape {
    static constexpr int H = N / 2 + 1;
    static constexpr long FS = long(H) * N * N;           // complex elements per half spectrum
    // y-pass / x-pass chunk of contiguous z values (128-byte runs of complex)
    static constexpr int TZ = (sizeof(R) == 4 ? 16 : 8) < N ? (sizeof(R) == 4 ? 16 : 8) : N;
    // zbin rows per block (a divisor of N)
    static constexpr int RBB = (N >= 256) ? 1 : (256 / N < N ? 256 / N : N);
    static constexpr int RBB_ = (N == 384) ? 1 : RBB;
    static constexpr int N2MAX = 3 * (N / 2) * (N / 2);
};

__device__ __forceinline__ int signed_index(int i, int N) { return i < N / 2 ? i : i - N; }


// Workgroups are dispatched round-robin over the 8 XCDs of the chip, each
// with its own L2.  xcd_block renumbers the nb blocks of a grid row so that
// every XCD works through one contiguous range of logical blocks.  The
// x-pass tiles read half cache lines (64 bytes) whose other halves belong to
// the neighbouring z chunk: in this order both halves are requested through
// the same L2 instead of being fetched from HBM twice.
__device__ __forceinline__ int xcd_block(int b, int nb) {
    const int x = b % 8, s = b / 8;
    const int q = nb / 8, r = nb % 8;
    return x * q + (x < r ? x : r) + s;
}

// Workgroup barrier for LDS hand-offs only: it waits for this wavefront's
// LDS operations (lgkmcnt) and nothing else.  __syncthreads makes every LDS
// write visible to the workgroup, and since global-to-LDS loads write LDS,
// it also waits for all of those in flight (vmcnt): a tile requested for
// the next term would have to land at the very next barrier.  With this
// barrier it stays in flight.  The memory clobber keeps the compiler from
// moving memory accesses across it; a caller that needs a global-to-LDS
// load to have landed waits for it explicitly.
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// Layout of the gradient fields U (written by ypass3, read by xprod): tiles
// of TZT z values, 128 bytes.  Element (kx, y, z) of a field sits at
//   ((y * (N / TZT) + z / TZT) * hs + kx) * TZT + z % TZT,
// hs = kx_sup + 1 the planes of the target's support (N/2 + 1 when it
// covers the lattice): the written and read part of a field is one
// contiguous block whatever the support.
// ypass3 writes whole 128-byte lines per (kx, y); the hs x TZT region
// that the xprod blocks of one (y, z tile) read together is contiguous.  At
// 512^3 the x pass reads this about twice as fast as the kx-major
// half-spectrum order, at 256^3 about as fast; 256- and 512-byte tiles and a
// y-major order measured no better.
template <typename R, int N> struct TTile {
    static constexpr int TZT0 = 128 / int(2 * sizeof(R));
    static constexpr int TZT = TZT0 < N ? TZT0 : N;
};
template <int N, int TZT>
__device__ __forceinline__ long t_offset(int kx, int y, int z, int hs) {
    return ((long(y) * (N / TZT) + z / TZT) * hs + kx) * TZT + z % TZT;
}

// Raw buffer loads of complex values.  The descriptor covers `bytes` bytes
// from a wave-uniform base; a load whose byte offset is at or past that
// count returns zero and makes no memory access (the buffer unit's range
// check), which is how known-zero elements are read without predication.
constexpr unsigned kBufOutside = 0x80000000u;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* base, unsigned bytes) {
    // third word 0x00020000: 32-bit data format, as the gfx9 family expects
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, int(bytes), 0x00020000);
}
typedef unsigned BufU2 __attribute__((ext_vector_type(2)));
typedef unsigned BufU4 __attribute__((ext_vector_type(4)));
template <typename C> __device__ __forceinline__ C buf_load(__amdgpu_buffer_rsrc_t rs, unsigned off);
template <> __device__ __forceinline__ float2 buf_load<float2>(__amdgpu_buffer_rsrc_t rs, unsigned off) {
    const BufU2 v = __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0);
    return make_float2(__uint_as_float(v.x), __uint_as_float(v.y));
}
template <> __device__ __forceinline__ double2 buf_load<double2>(__amdgpu_buffer_rsrc_t rs, unsigned off) {
    const BufU4 v = __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0);
    return make_double2(__hiloint2double(int(v.y), int(v.x)), __hiloint2double(int(v.w), int(v.z)));
}

// ----------------------------------------------------------------------------
// White noise: Philox4x64-10 (Salmon et al., SC'11) + Box-Muller cosine branch.
// The binary64 ln and cos below follow an explicit operation sequence with no
// contraction, so that the deviates are reproducible bit for bit by any
// implementation of the same sequence.
// ----------------------------------------------------------------------------
struct Philox4x64 {
    static constexpr uint64_t M0 = 0xD2E7470EE14C6C93ull;
    static constexpr uint64_t M1 = 0xCA5A826395121157ull;
    static constexpr uint64_t W0 = 0x9E3779B97F4A7C15ull;
    static constexpr uint64_t W1 = 0xBB67AE8584CAA73Bull;
};

__device__ __forceinline__ void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += Philox4x64::W0;
            k1 += Philox4x64::W1;
        }
        const uint64_t hi0 = __umul64hi(Philox4x64::M0, c[0]);
        const uint64_t lo0 = Philox4x64::M0 * c[0];
        const uint64_t hi1 = __umul64hi(Philox4x64::M1, c[2]);
        const uint64_t lo1 = Philox4x64::M1 * c[2];
        const uint64_t n0 = hi1 ^ c[1] ^ k0;
        const uint64_t n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
    }
}

#pragma clang fp contract(off)
__device__ __noinline__ double spec_ln(double u) {
    constexpr double LN2 = 0.6931471805599453;
    constexpr double SQRT2 = 1.4142135623730951;
    constexpr double C[13] = {1.0 / 1.0,  1.0 / 3.0,  1.0 / 5.0,  1.0 / 7.0,  1.0 / 9.0,
                              1.0 / 11.0, 1.0 / 13.0, 1.0 / 15.0, 1.0 / 17.0, 1.0 / 19.0,
                              1.0 / 21.0, 1.0 / 23.0, 1.0 / 25.0};
    int e0;
    const double m0 = frexp(u, &e0);
    double m = m0 * 2.0;
    double e = (double)(e0 - 1);
    if (m > SQRT2) {
        m = m * 0.5;
        e = e + 1.0;
    }
    const double s = (m - 1.0) / (m + 1.0);
    const double z = s * s;
    double p = C[12];
    for (int k = 11; k >= 0; --k) {
        p = p * z;
        p = p + C[k];
    }
    const double t = s + s;
    const double a = e * LN2;
    const double b = t * p;
    return a + b;
}

__device__ __noinline__ double spec_cos2pi(double u) {
    constexpr double PIO2 = 1.5707963267948966;
    constexpr double CC[10] = {1.0,
                               -1.0 / 2.0,
                               1.0 / 24.0,
                               -1.0 / 720.0,
                               1.0 / 40320.0,
                               -1.0 / 3628800.0,
                               1.0 / 479001600.0,
                               -1.0 / 87178291200.0,
                               1.0 / 20922789888000.0,
                               -1.0 / 6402373705728000.0};
    constexpr double SC[10] = {1.0,
                               -1.0 / 6.0,
                               1.0 / 120.0,
                               -1.0 / 5040.0,
                               1.0 / 362880.0,
                               -1.0 / 39916800.0,
                               1.0 / 6227020800.0,
                               -1.0 / 1307674368000.0,
                               1.0 / 355687428096000.0,
                               -1.0 / 121645100408832000.0};
    const double t = u * 4.0;
    const double q = floor(t);
    const double f = t - q;
    const bool hi = f > 0.5;
    const double g = hi ? 1.0 - f : f;
    const double x = g * PIO2;
    const double z = x * x;
    double c = CC[9];
    for (int k = 8; k >= 0; --k) {
        c = c * z;
        c = c + CC[k];
    }
    double sp = SC[9];
    for (int k = 8; k >= 0; --k) {
        sp = sp * z;
        sp = sp + SC[k];
    }
    const double sn = x * sp;
    const double cf = hi ? sn : c;
    const double sf = hi ? c : sn;
    const int qi = (int)q;
    return qi == 0 ? cf : (qi == 1 ? -sf : (qi == 2 ? -cf : sf));
}

__device__ __noinline__ double spec_normal(uint64_t w0, uint64_t w1) {
    const double u1 = ((double)(w0 >> 12) * 2.0 + 1.0) * 0x1.0p-53;
    const double u2 = ((double)(w1 >> 12) * 2.0 + 1.0) * 0x1.0p-53;
    const double l = spec_ln(u1);
    const double r = sqrt(l * -2.0);
    return r * spec_cos2pi(u2);
}
#pragma clang fp contract(fast)

template <typename R>
__global__ __launch_bounds__(256) void k_noise(R* __restrict__ out, long total, uint64_t seed) {
    const long s = long(blockIdx.x) * 256 + threadIdx.x;
    if (s >= total) return;
    uint64_t c[4] = {(uint64_t)s, 0ull, 0ull, 0ull};
    philox4x64_10(c, seed, 0ull);
    out[s] = (R)spec_normal(c[0], c[1]);
}

// ----------------------------------------------------------------------------
// Pass tiles.  Every transform below is the two-phase register FFT of
// sigw_fft.hpp: one register DFT of size R1, one LDS transpose, one register
// DFT of size R2 (N = R1 R2).
// ----------------------------------------------------------------------------
template <int N> struct TPConst {
    static constexpr int R1 = TwoPhase<N>::R1;
    static constexpr int R2 = N / R1;
    static constexpr int RMIN = R1 < R2 ? R1 : R2;
    static constexpr int RMAX = R1 > R2 ? R1 : R2;
};

template <int A, int B> struct CMin { static constexpr int v = A < B ? A : B; };
template <int A, int B> struct CMax { static constexpr int v = A > B ? A : B; };
constexpr int pow2_floor(long x) {
    int p = 1;
    while (2L * p <= x) p *= 2;
    return p;
}

// z pass: complex DFT along contiguous rows, in place.  RB rows per block.
template <typename R, int N> struct ZCfg {
    using C = typename CplxOf<R>::T;
    static constexpr int NT = 256;
    static constexpr int RB0 = CMax<1, NT / TPConst<N>::RMIN>::v;
    // keep the transpose tile at or below 64 KB (a power of two, so it divides N)
    static constexpr long ROWB = long(TPLayout<N, 1, false>::size) * long(sizeof(C));
    static constexpr int RB = pow2_floor(RB0 * ROWB > 65536 ? 65536 / ROWB : RB0);
};

template <typename R, int N, int SIGN>
__global__ __launch_bounds__(256) void k_zpass(typename CplxOf<R>::T* __restrict__ data, long n_rows,
                                               const typename CplxOf<R>::T* __restrict__ tw) {
    using C = typename CplxOf<R>::T;
    constexpr int RB = ZCfg<R, N>::RB;
    constexpr int NT = ZCfg<R, N>::NT;
    __shared__ C lds[TPLayout<N, RB, false>::size];
    const int tid = threadIdx.x;
    const long row0 = long(blockIdx.x) * RB;
    C* base = data + row0 * N;
    auto ld = [&](int line, int n) -> C {
        return (row0 + line < n_rows) ? base[long(line) * N + n] : cmk<C>(R(0), R(0));
    };
    auto st = [&](int line, int k, C v) {
        if (row0 + line < n_rows) base[long(line) * N + k] = v;
    };
    tp_phase1<C, N, SIGN, RB, NT, false>(ld, lds, tw, tid);
    __syncthreads();
    tp_phase2<C, N, SIGN, RB, NT, false>(st, lds, tid);
}

// y pass: complex DFT along y of tiles (field, kx plane, z chunk), in place.
template <typename R, int N> struct YCfg {
    static constexpr int TZ = Shape<R, N>::TZ;
    static constexpr int NT = CMin<256, CMax<64, TZ * TPConst<N>::RMIN>::v>::v;
    // first radix of ypass3: from 384^3 on (FP32) a larger one leaves one
    // phase-1 item per thread (TZ R2 = NT), so the W tile stays in registers
    // for both of its rounds instead of being read twice
    static constexpr int R1_3 = (sizeof(R) == 4 && N >= 384) ? N * TZ / NT : 0;
};

template <typename R, int N, int SIGN>
__global__ __launch_bounds__(256) void k_ypass(typename CplxOf<R>::T* __restrict__ data, long field_stride,
                                               int n_planes, long batch_stride,
                                               const typename CplxOf<R>::T* __restrict__ tw) {
    using C = typename CplxOf<R>::T;
    constexpr int TZ = YCfg<R, N>::TZ;
    constexpr int NT = YCfg<R, N>::NT;
    constexpr int NZC = N / TZ;
    __shared__ C lds[TPLayout<N, TZ, true>::size];
    const int tid = threadIdx.x;
    const long b = blockIdx.x;
    const int zc = int(b % NZC);
    const long fp = b / NZC;
    const int kx = int(fp % n_planes);
    const long f = fp / n_planes;
    C* base = data + blockIdx.y * batch_stride + f * field_stride + long(kx) * N * N + zc * TZ;
    auto ld = [&](int zz, int y) -> C { return base[long(y) * N + zz]; };
    auto st = [&](int zz, int y, C v) { base[long(y) * N + zz] = v; };
    tp_phase1<C, N, SIGN, TZ, NT, true>(ld, lds, tw, tid);
    __syncthreads();
    tp_phase2<C, N, SIGN, TZ, NT, true>(st, lds, tid);
}

// x pass, real -> half (forward).  Tile (y, z chunk); the z pairs (2p, 2p+1)
// ride as the real and imaginary parts of one complex line of length N.
template <typename R, int N> struct XCfg {
    static constexpr int TZ = Shape<R, N>::TZ;
    static constexpr int P = TZ / 2;
    static constexpr int NT = CMin<256, CMax<64, P * TPConst<N>::RMAX>::v>::v;
};

template <typename R, int N>
__global__ __launch_bounds__(256) void k_xpass_r2c(const R* __restrict__ in, typename CplxOf<R>::T* __restrict__ out,
                                                   const typename CplxOf<R>::T* __restrict__ tw) {
    using C = typename CplxOf<R>::T;
    constexpr int TZ = XCfg<R, N>::TZ;
    constexpr int P = XCfg<R, N>::P;
    constexpr int NT = XCfg<R, N>::NT;
    constexpr int NZC = N / TZ;
    constexpr int H = N / 2 + 1;
    constexpr int LS = N + 1;
    __shared__ C lds[TPLayout<N, P, true>::size];
    __shared__ C zb[P * LS];
    const int tid = threadIdx.x;
    const int bl = xcd_block(int(blockIdx.x), int(gridDim.x));
    const int zc = bl % NZC;
    const int y = bl / NZC;
    const int z0 = zc * TZ;
    const C* inc = reinterpret_cast<const C*>(in);
    auto ld = [&](int p, int x) -> C { return inc[((long(x) * N + y) * N + z0) / 2 + p]; };
    auto st = [&](int p, int k, C v) { zb[p * LS + k] = v; };
    tp_phase1<C, N, -1, P, NT, true>(ld, lds, tw, tid);
    __syncthreads();
    tp_phase2<C, N, -1, P, NT, true>(st, lds, tid);
    __syncthreads();
    for (int e = tid; e < H * P; e += NT) {
        const int k = e / P, p = e % P;
        const C zk = zb[p * LS + k];
        const C zm = zb[p * LS + ((N - k) % N)];
        const C a = cmk<C>(R(0.5) * (zk.x + zm.x), R(0.5) * (zk.y - zm.y));
        const C bb = cmk<C>(R(0.5) * (zk.y + zm.y), R(-0.5) * (zk.x - zm.x));
        C* o = out + (long(k) * N + y) * N + z0 + 2 * p;
        o[0] = a;
        o[1] = bb;
    }
}

// Hermitian-extended pair line for the inverse along x: element n of line p
// is X_a[n] + i X_b[n] (n <= N/2) or conj(X_a[N-n]) + i conj(X_b[N-n]), with
// X_a, X_b the z = 2p and 2p+1 columns of the half spectrum at (y, z0);
// the imaginary parts at kx = 0 and N/2 are dropped (real-input convention).
// With grad set, both columns are first multiplied by i qt_x(kx),
// qt_x = k_F n_x (zero at kx = 0 and on the Nyquist plane).  Branch free, so
// lines with and without the gradient can share a wavefront.
template <typename C, int N>
__device__ __forceinline__ C herm_pair(const C* __restrict__ col, int n, bool grad = false,
                                       decltype(C::x) k_F = 0) {
    using R = decltype(C::x);
    const int k = n <= N / 2 ? n : N - n;
    const C* src = col + long(k) * N * N;
    C a = src[0], b = src[1];
    const bool edge = (k == 0 || k == N / 2);
    const R q = (grad && !edge) ? k_F * R(k) : R(0);   // i q multiplier on the gradient line
    const R keep = grad ? R(0) : R(1);
    const R ky = edge ? R(0) : keep;                    // imaginary parts kept off the edges
    a = cmk<C>(keep * a.x - q * a.y, ky * a.y + q * a.x);
    b = cmk<C>(keep * b.x - q * b.y, ky * b.y + q * b.x);
    return n <= N / 2 ? cmk<C>(a.x - b.y, a.y + b.x) : cmk<C>(a.x + b.y, b.x - a.y);
}

// x pass, half -> real (inverse).
template <typename R, int N>
__global__ __launch_bounds__(256) void k_xpass_c2r(const typename CplxOf<R>::T* __restrict__ in, R* __restrict__ out,
                                                   const typename CplxOf<R>::T* __restrict__ tw) {
    using C = typename CplxOf<R>::T;
    constexpr int TZ = XCfg<R, N>::TZ;
    constexpr int P = XCfg<R, N>::P;
    constexpr int NT = XCfg<R, N>::NT;
    constexpr int NZC = N / TZ;
    __shared__ C lds[TPLayout<N, P, true>::size];
    const int tid = threadIdx.x;
    const int bl = xcd_block(int(blockIdx.x), int(gridDim.x));
    const int zc = bl % NZC;
    const int y = bl / NZC;
    const int z0 = zc * TZ;
    C* outc = reinterpret_cast<C*>(out);
    const C* col0 = in + long(y) * N + z0;
    auto ld = [&](int p, int n) -> C { return herm_pair<C, N>(col0 + 2 * p, n); };
    auto st = [&](int p, int x, C v) { outc[((long(x) * N + y) * N + z0) / 2 + p] = v; };
    tp_phase1<C, N, +1, P, NT, true>(ld, lds, tw, tid);
    __syncthreads();
    tp_phase2<C, N, +1, P, NT, true>(st, lds, tid);
}

// ----------------------------------------------------------------------------
// Spectral filter and field maps.
// ----------------------------------------------------------------------------
template <typename R, int N>
__global__ __launch_bounds__(256) void k_filter(typename CplxOf<R>::T* __restrict__ half, const double* __restrict__ amp) {
    using C = typename CplxOf<R>::T;
    constexpr long FS = Shape<R, N>::FS;
    const long i = long(blockIdx.x) * 256 + threadIdx.x;
    if (i >= FS) return;
    const int kz = int(i % N);
    const int ky = int((i / N) % N);
    const int kx = int(i / (long(N) * N));
    const int nx = signed_index(kx, N), ny = signed_index(ky, N), nz = signed_index(kz, N);
    const R a = (R)amp[nx * nx + ny * ny + nz * nz];
    C v = half[i];
    half[i] = cmk<C>(v.x * a, v.y * a);
}

// Spectral Laplacian of a half spectrum, times a constant: X(n) *= c |n|^2.
template <typename R, int N>
__global__ __launch_bounds__(256) void k_laplacian(typename CplxOf<R>::T* __restrict__ half, double c) {
    using C = typename CplxOf<R>::T;
    constexpr long FS = Shape<R, N>::FS;
    const long i = long(blockIdx.x) * 256 + threadIdx.x;
    if (i >= FS) return;
    const int kz = int(i % N);
    const int ky = int((i / N) % N);
    const int kx = int(i / (long(N) * N));
    const int nx = signed_index(kx, N), ny = signed_index(ky, N), nz = signed_index(kz, N);
    const R a = (R)(c * double(nx * nx + ny * ny + nz * nz));
    C v = half[i];
    half[i] = cmk<C>(v.x * a, v.y * a);
}

template <typename R>
__global__ __launch_bounds__(256) void k_square(const R* __restrict__ in, R* __restrict__ out, long total) {
    const long i = long(blockIdx.x) * 256 + threadIdx.x;
    if (i >= total) return;
    const double v = (double)in[i];
    out[i] = (R)(v * v);
}

// zeta = zeta_g + l1 + zeta_g l2 (the two Laplacian terms of the non-local
// map, their coefficients already applied), in FP64
template <typename R>
__global__ __launch_bounds__(256) void k_nonlocal_combine(const R* __restrict__ zg, const R* __restrict__ l1,
                                                          const R* __restrict__ l2, R* __restrict__ out,
                                                          long total) {
    const long i = long(blockIdx.x) * 256 + threadIdx.x;
    if (i >= total) return;
    const double z = (double)zg[i];
    out[i] = (R)(z + (double)l1[i] + z * (double)l2[i]);
}

template <typename R>
__global__ __launch_bounds__(256) void k_sumsq_partial(const R* __restrict__ x, long total, double* __restrict__ part) {
    __shared__ double red[256];
    const int tid = threadIdx.x;
    const long per = (total + gridDim.x - 1) / gridDim.x;
    const long lo = long(blockIdx.x) * per;
    const long hi = (lo + per < total) ? lo + per : total;
    double acc = 0.0;
    for (long i = lo + tid; i < hi; i += 256) {
        const double v = (double)x[i];
        acc += v * v;
    }
    red[tid] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) red[tid] += red[tid + s];
        __syncthreads();
    }
    if (tid == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_reduce_sum(const double* __restrict__ part, int n, double* __restrict__ out) {
    __shared__ double red[256];
    const int tid = threadIdx.x;
    double acc = 0.0;
    for (int i = tid; i < n; i += 256) acc += part[i];
    red[tid] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) red[tid] += red[tid + s];
        __syncthreads();
    }
    if (tid == 0) out[0] = red[0];
}

template <typename R>
__global__ __launch_bounds__(256) void k_map_scale(const R* __restrict__ in, R* __restrict__ out, long total,
                                                   const double* __restrict__ sum_sq, MapParams mp, double scale) {
    const long i = long(blockIdx.x) * 256 + threadIdx.x;
    if (i >= total) return;
    const double zg = (double)in[i];
    double z;
    if (mp.kind == 1) {
        const double m2 = sum_sq[0] / (double)total;
        z = zg + mp.F_NL * (zg * zg - m2) + mp.G_NL * zg * zg * zg;
    } else if (mp.kind == 2) {
        double a = 1.0 - mp.beta * zg;
        a = a > mp.clip ? a : mp.clip;
        z = -log(a) / mp.beta;
    } else {
        z = zg;
    }
    out[i] = (R)(z * scale);
}

// ----------------------------------------------------------------------------
// Half spectrum of an N grid from half spectra of a larger n_src grid (the
// same box): every mode of the N grid, by signed index, copied from the
// source.  Used for targets whose convolution fits a smaller grid exactly.
// ----------------------------------------------------------------------------
template <typename R, int N>
__global__ __launch_bounds__(256) void k_restrict(const typename CplxOf<R>::T* __restrict__ src, int n_src,
                                                  const int* __restrict__ sel,
                                                  typename CplxOf<R>::T* __restrict__ dst) {
    constexpr long FS = Shape<R, N>::FS;
    const long i = long(blockIdx.x) * 256 + threadIdx.x;
    if (i >= FS) return;
    const int kx = int(i / (long(N) * N));
    const int ky = int((i / N) % N), kz = int(i % N);
    const int ny = signed_index(ky, N), nz = signed_index(kz, N);
    const long sy = ny < 0 ? ny + n_src : ny, sz = nz < 0 ? nz + n_src : nz;
    const long fs_src = long(n_src / 2 + 1) * n_src * n_src;
    dst[long(blockIdx.y) * FS + i] = src[long(sel[blockIdx.y]) * fs_src + (long(kx) * n_src + sy) * n_src + sz];
}

// ----------------------------------------------------------------------------
// Per-target lookup tables over integer |n|^2.
// ----------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_lut(int n2max, double k_F, double k_target, double k_lo, double k_hi,
                                             const double* __restrict__ edges, int n_modes,
                                             int16_t* __restrict__ lut_u, uint8_t* __restrict__ lut_shell) {
    const int n2 = blockIdx.x * 256 + threadIdx.x;
    if (n2 > n2max) return;
    const double rt = sqrt((double)n2);
    const double u = k_F * rt / k_target;
    int idx = -1;
    if (u >= edges[0] && u < edges[n_modes]) {
        int lo = 0, hi = n_modes;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (edges[mid] <= u) lo = mid;
            else hi = mid;
        }
        idx = lo;
    }
    lut_u[n2] = (int16_t)idx;
    const double k = k_F * rt;
    lut_shell[n2] = (n2 > 0 && k >= k_lo && k < k_hi) ? 1 : 0;
}

// ----------------------------------------------------------------------------
// gen_z: Fourier weighting fused into the first inverse pass (along z).
// Block = RB rows (kx, ky).  Phase-1 items are (row, t); each holds the R1
// elements kz = t + R2 m of its row (Phi_hat / V and the u-interval) in
// registers for the whole loop over kept terms a, and forms two fields:
//   W_a = IDFT_z( phi_a(u) Phi_hat / V ),  Z_a = IDFT_z( i qt_z phi_a(u) Phi_hat / V ).
// The x and y gradients are applied later (i qt_y before the y transform,
// i qt_x in the x pass), so two fields per term cross HBM here, not three.
// Rows outside the support (nx^2 + ny^2 > n2_sup) are zero for every term:
// they are neither read nor written (ypass3 reads them as zeros).  Grid x =
// term groups of tg terms x planes kx <= kx_sup x c0 row blocks, c0 the live
// row blocks of plane 0 (the most of any plane); block j of plane kx takes
// that plane's j-th live row block, if it has one.  A small support leaves
// few live row blocks, and splitting the terms over blocks keeps the chip
// busy (Phi_hat is then read once per group, a small fraction of the
// writes).
// ----------------------------------------------------------------------------
// Largest y >= 0 with y^2 <= v (v >= 0), at most N/2: the largest live |ny|
// of a row set bounded by ny^2 <= v.
template <int N> __host__ __device__ inline int ylim_of(int v) {
    int r = int(sqrt(double(v)));
    while (r > 0 && r * r > v) --r;
    while ((r + 1) * (r + 1) <= v) ++r;
    return r < N / 2 ? r : N / 2;
}
// Row blocks (RB consecutive ky) of one kx plane that hold live rows, the
// live rows being ky <= ylim and ky >= N - ylim: the first lc blocks and the
// last uc, or all N/RB when the two runs meet.
template <int N, int RB> __host__ __device__ inline int live_row_blocks(int ylim) {
    const int lc = ylim / RB + 1;
    const int uc = ylim > 0 ? N / RB - (N - ylim) / RB : 0;
    return lc + uc >= N / RB ? N / RB : lc + uc;
}
template <int N, int RB> __host__ __device__ inline int live_row_block(int ylim, int j) {
    const int lc = ylim / RB + 1;
    const int uc = ylim > 0 ? N / RB - (N - ylim) / RB : 0;
    if (lc + uc >= N / RB) return j;
    return j < lc ? j : N / RB - uc + (j - lc);
}

template <typename R, int N> struct GCfg {
    static constexpr int R1 = TPConst<N>::R1;
    static constexpr int R2 = TPConst<N>::R2;
    static constexpr int RB0 = (sizeof(R) == 4 ? 2048 : 1024) / N;
    static constexpr int RB = pow2_floor(CMin<CMax<1, RB0>::v, N>::v);
    static constexpr int NT = CMin<256, CMax<64, RB * R2>::v>::v;
};

template <typename R, int N>
__global__ __launch_bounds__(256) void k_gen_z(const typename CplxOf<R>::T* __restrict__ phi_hat_all,
                                               const int* __restrict__ sel, const int16_t* __restrict__ lut_u,
                                               const R* __restrict__ phi_tab, int n_alpha, int a0, int na, R k_F,
                                               R inv_V, typename CplxOf<R>::T* __restrict__ S_all, long s_stride,
                                               int n2_sup, int c0, int nrb, int tg,
                                               const typename CplxOf<R>::T* __restrict__ tw) {
    using C = typename CplxOf<R>::T;
    using G = GCfg<R, N>;
    constexpr int RB = G::RB, NT = G::NT, R1 = G::R1, R2 = G::R2;
    constexpr int NL = 2 * RB;
    using Lay = TPLayout<N, NL, false>;
    constexpr long FS = Shape<R, N>::FS;
    constexpr int ITEMS = RB * R2;
    constexpr int PER = (ITEMS + NT - 1) / NT;
    __shared__ C lds[Lay::size];
    static_assert(N % RB == 0 && RB <= 32, "the rows of a block share one kx plane");
    const int tid = threadIdx.x;
    const int rem = int(blockIdx.x % nrb);
    const int kxb = rem / c0, jb = rem % c0;
    const int ylb = ylim_of<N>(n2_sup - kxb * kxb);
    if (jb >= live_row_blocks<N, RB>(ylb)) return;           // uniform over the block
    const long row0 = long(kxb) * N + long(live_row_block<N, RB>(ylb, jb)) * RB;
    const int ab = a0 + int(blockIdx.x / nrb) * tg;       // this block's terms [ab, ae)
    const int ae = ab + tg < a0 + na ? ab + tg : a0 + na;
    // rows of this block inside the support: bit row of live
    unsigned live = 0;
    {
        const int nx = signed_index(int(row0 / N), N);
        const int lim = n2_sup - nx * nx;
#pragma unroll
        for (int row = 0; row < RB; ++row) {
            const int ny = signed_index(int((row0 + row) % N), N);
            if (ny * ny <= lim) live |= 1u << row;
        }
    }
    if (live == 0) return;                                  // uniform over the block
    // FULL: every row of the block is live (the common case), and the row
    // predicates drop out of the compiled form
    auto run = [&](auto full) {
    constexpr bool FULL = decltype(full)::value;
    // batch member blockIdx.y works on the realisation in slot sel[blockIdx.y]
    const C* phi_hat = phi_hat_all + long(sel[blockIdx.y]) * FS;
    C* T = S_all + blockIdx.y * s_stride;
    C ph[PER][R1];
    int16_t idx[PER][R1];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int w = tid + i * NT;
        const bool inr = (ITEMS % NT == 0) || w < ITEMS;
        const int row = inr ? w / R2 : 0;
        const bool ok = inr && (FULL || ((live >> row) & 1u));
        const int t = ok ? w % R2 : 0;
        const long r = row0 + row;
        const int kx = int(r / N), ky = int(r % N);
        const int nx = signed_index(kx, N), ny = signed_index(ky, N);
#pragma unroll
        for (int m = 0; m < R1; ++m) {
            const int kz = t + R2 * m;
            const int nz = signed_index(kz, N);
            const C v = ok ? phi_hat[r * N + kz] : cmk<C>(R(0), R(0));
            ph[i][m] = cmk<C>(v.x * inv_V, v.y * inv_V);
            idx[i][m] = ok ? lut_u[nx * nx + ny * ny + nz * nz] : int16_t(-1);
        }
    }
    for (int a = ab; a < ae; ++a) {
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int w = tid + i * NT;
            if ((ITEMS % NT == 0) || w < ITEMS) {
                const int row = w / R2, t = w % R2;
                C v[R1];
#pragma unroll
                for (int m = 0; m < R1; ++m) {
                    const R wgt = idx[i][m] >= 0 ? phi_tab[idx[i][m] * n_alpha + a] : R(0);
                    v[m] = cmk<C>(ph[i][m].x * wgt, ph[i][m].y * wgt);
                }
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    C f[R1];
#pragma unroll
                    for (int m = 0; m < R1; ++m) {
                        if (j == 0) {
                            f[m] = v[m];
                        } else {
                            const int nz = signed_index(t + R2 * m, N);
                            const R q = (nz == -N / 2) ? R(0) : k_F * R(nz);
                            f[m] = cmk<C>(-q * v[m].y, q * v[m].x);   // i q_z v
                        }
                    }
                    reg_dft<R1, +1>(f);
#pragma unroll
                    for (int k1 = 0; k1 < R1; ++k1) {
                        C o = f[k1];
                        if (k1 > 0) o = cmul(o, tw_at<+1, N>(tw, t * k1));
                        lds[Lay::at(j * RB + row, k1, t)] = o;
                    }
                }
            }
        }
        __syncthreads();
        const long fbase = long(2 * (a - a0)) * FS;
        auto st = [&](int line, int kz, C v) {
            const int j = line / RB, row = line % RB;
            if (FULL || ((live >> row) & 1u)) T[fbase + long(j) * FS + (row0 + row) * N + kz] = v;
        };
        tp_phase2<C, N, +1, NL, NT, false>(st, lds, tid);
        __syncthreads();
    }
    };
    constexpr unsigned kAll = RB == 32 ? 0xffffffffu : (1u << RB) - 1u;
    if (live == kAll) run(std::true_type{});
    else run(std::false_type{});
}

// ----------------------------------------------------------------------------
// ypass3: inverse DFT along y that expands the two z-transformed fields of
// each term into its three gradient fields:
//   U_x = i qt_x IDFT_y(W_a),  U_y = IDFT_y(i qt_y W_a),  U_z = IDFT_y(Z_a)
// (qt_x is uniform over a block's kx plane, so its factor costs nothing
// here and leaves the x pass a uniform Hermitian extension).  Tile (term,
// kx plane, z chunk); the three outputs are transformed one after another
// through the same LDS tile and stored in the x-pass tile layout (t_offset).
// The grid covers the planes kx < hs = kx_sup + 1 only; rows of the input
// outside the support (nx^2 + ny^2 > n2_sup) were not written by gen_z and
// are read as zeros.
// ----------------------------------------------------------------------------
template <typename R, int N>
__global__ __launch_bounds__(256) void k_ypass3(const typename CplxOf<R>::T* __restrict__ S_all, long s_stride,
                                                typename CplxOf<R>::T* __restrict__ T_all, long t_stride, R k_F,
                                                int n2_sup, int hs,
                                                const typename CplxOf<R>::T* __restrict__ tw) {
    using C = typename CplxOf<R>::T;
    constexpr int TZ = YCfg<R, N>::TZ;
    constexpr int NT = YCfg<R, N>::NT;
    constexpr int NZC = N / TZ;
    constexpr int H = N / 2 + 1;
    constexpr long FS = Shape<R, N>::FS;
    constexpr int TZT = TTile<R, N>::TZT;
    static_assert(TZT % TZ == 0, "a y-pass chunk lies inside one field tile");
    constexpr int YR1 = YCfg<R, N>::R1_3;
    using Lay = TPLayout<N, TZ, true, YR1>;
    constexpr int R1 = Lay::R1, R2 = Lay::R2;
    constexpr int ITEMS = TZ * R2;
    constexpr int PER = (ITEMS + NT - 1) / NT;
    __shared__ C lds[Lay::size];
    __shared__ C twl[N];
    const int tid = threadIdx.x;
    stage_twiddles<C, N, NT>(twl, tw, tid);
    // consecutive z chunks of a (term, kx) plane share an XCD and its L2,
    // which keeps the DRAM pages of that plane's rows together (measured
    // faster)
    const long b = xcd_block(int(blockIdx.x), int(gridDim.x));
    const int zc = int(b % NZC);
    const long fp = b / NZC;
    const int kx = int(fp % hs);
    const long al = fp / hs;
    const long off = long(kx) * N * N + zc * TZ;
    const C* S = S_all + blockIdx.y * s_stride;
    C* T = T_all + blockIdx.y * t_stride;
    const C* w = S + 2 * al * FS + off;
    const C* z = w + FS;
    // Rows of the input outside the support read as zeros.  The live rows
    // are ny in [-ylim, ylim] (lim >= 0 on the planes kx <= kx_sup): the
    // prefix y <= ylim and the suffix y >= N - ylim.  Descriptor lo covers
    // the prefix from the plane's start, descriptor hi the suffix from its
    // first row; the buffer range check returns zeros for every dead row (an
    // offset below the suffix wraps to a large unsigned value, and so does
    // kBufOutside for items past the tile), so the loads carry no
    // per-element predicate.
    const int lim = n2_sup - kx * kx;
    int ylim = int(sqrtf(float(lim)));
    while (ylim > 0 && ylim * ylim > lim) --ylim;
    while ((ylim + 1) * (ylim + 1) <= lim) ++ylim;
    ylim = ylim < N / 2 ? ylim : N / 2;
    static_assert(long(N) * N * sizeof(C) < kBufOutside / 2, "plane offsets fit the buffer range");
    constexpr int RowB = N * int(sizeof(C));
    const auto zlo = buf_rsrc(z, unsigned((ylim + 1) * RowB));
    const auto wlo = buf_rsrc(w, unsigned((ylim + 1) * RowB));
    const auto zhi = buf_rsrc(z + long(N - ylim) * N, unsigned(ylim * RowB));
    const auto whi = buf_rsrc(w + long(N - ylim) * N, unsigned(ylim * RowB));
    // element (row t + R2 m, z line) of this lane; lane_off = (t N + line) * sizeof(C)
    auto load_row = [&](const __amdgpu_buffer_rsrc_t& lo, const __amdgpu_buffer_rsrc_t& hi, unsigned lane_off,
                        int t, int m) -> C {
        const unsigned o = lane_off + unsigned(R2 * m * RowB);
        const unsigned oh = o - unsigned((N - ylim) * RowB);
        if (R2 * (m + 1) <= N / 2) return buf_load<C>(lo, o);     // lower half for every t
        if (R2 * m >= N / 2) return buf_load<C>(hi, oh);          // upper half for every t
        return (t + R2 * m < N / 2) ? buf_load<C>(lo, o) : buf_load<C>(hi, oh);
    };
    const R qx = (kx == N / 2) ? R(0) : k_F * R(kx);     // qt_x of this plane
    // the W tile feeds U_x and U_y: with one phase-1 item per thread it is
    // read once, into registers (line tid % TZ, elements tid / TZ + R2 m);
    // with more, registers are too scarce and U_y reads it again
    constexpr bool KEEP = PER == 1;
    C wr[1][R1];
    C zr[R1];
    if constexpr (KEEP) {
        // Z first, then W: the U_z round runs first and waits only for Z,
        // while the W loads stay in flight behind it
        const int it = tid;
        const bool ok = (ITEMS % NT == 0) || it < ITEMS;
        const int line = it % TZ, t = it / TZ;
        const unsigned lane_off = ok ? unsigned((t * N + line) * int(sizeof(C))) : kBufOutside;
#pragma unroll
        for (int m = 0; m < R1; ++m) zr[m] = load_row(zlo, zhi, lane_off, t, m);
#pragma unroll
        for (int m = 0; m < R1; ++m) wr[0][m] = load_row(wlo, whi, lane_off, t, m);
    }
    __syncthreads();                                        // twl
#pragma unroll
    for (int jj = 0; jj < 3; ++jj) {
        const int j = KEEP ? (jj + 2) % 3 : jj;             // rounds U_z, U_x, U_y when W is kept
        if constexpr (KEEP) {
            const int it = tid;
            if ((ITEMS % NT == 0) || it < ITEMS) {
                const int line = it % TZ, t = it / TZ;
                C v[R1];
#pragma unroll
                for (int m = 0; m < R1; ++m) {
                    const int yy = t + R2 * m;
                    if (j == 2) {
                        v[m] = zr[m];
                    } else {
                        R q = qx;
                        if (j == 1) {
                            const int ny = signed_index(yy, N);
                            q = (ny == -N / 2) ? R(0) : k_F * R(ny);
                        }
                        v[m] = cmk<C>(-q * wr[0][m].y, q * wr[0][m].x);
                    }
                }
                tp_phase1_item<C, N, +1, TZ, true, YR1>(v, line, t, lds, twl);
            }
        } else {
            auto ld = [&](int zz, int t, int m) -> C {
                const int yy = t + R2 * m;
                const unsigned lane_off = unsigned((t * N + zz) * int(sizeof(C)));
                C v = j == 2 ? load_row(zlo, zhi, lane_off, t, m) : load_row(wlo, whi, lane_off, t, m);
                if (j < 2) {
                    R q = qx;
                    if (j == 1) {
                        const int ny = signed_index(yy, N);
                        q = (ny == -N / 2) ? R(0) : k_F * R(ny);
                    }
                    v = cmk<C>(-q * v.y, q * v.x);
                }
                return v;
            };
            tp_phase1_tm<C, N, +1, TZ, NT, true, YR1>(ld, lds, twl, tid);
        }
        __syncthreads();
        C* dst = T + (3 * al + j) * FS;
        auto st = [&](int zz, int y, C v) { dst[t_offset<N, TZT>(kx, y, zc * TZ + zz, hs)] = v; };
        tp_phase2<C, N, +1, TZ, NT, true, YR1>(st, lds, tid);
        __syncthreads();
    }
}

// ----------------------------------------------------------------------------
// xprod: last inverse pass (x, complex -> real) + products + first forward
// pass (x, real -> complex).  Block = (y, z chunk of TZX).  Q stays in
// registers across all kept terms.
//
// Per term the raw tile (3 fields x (N/2+1) kx x TZX z values) is loaded
// once, coalesced, straight from global memory into LDS by the gfx950
// global-to-LDS loads (no registers involved).  The tile of term a+1 is
// requested as soon as phase 1 of term a has read the buffer, so it is in
// flight during phase 2 and the products; one buffer per block keeps the
// LDS at about 52 KB, three blocks per CU, which hides more latency than a
// second buffer would (measured).  The Hermitian extension of the x lines
// is applied when phase 1 reads the tile back (the gradient factors were
// applied by the earlier passes).  Planes kx > kx_sup are outside the
// support of every term: their part of the tile is zeroed once and never
// loaded.
// ----------------------------------------------------------------------------
// x-pass schedule: TZX z values (TZX/2 pairs) per block, a part of one
// gradient-field tile; threads: a divisor of the N TZX/2 point pairs, at
// most 256.  LDS: raw tile, phase-1 transpose / G lines, twiddle copy.
template <typename R, int N, int TZX_> struct XShape {
    static constexpr int TZX = TZX_ < N ? TZX_ : N;
    static constexpr int PX = TZX / 2;
    static constexpr int NPP = N * PX;
    static constexpr int NTX = NPP <= 256 ? NPP : (NPP % 256 == 0 ? 256 : (NPP % 192 == 0 ? 192 : 128));
    static constexpr int PPX = NPP / NTX;                 // point pairs per thread
    static_assert(NTX * PPX == NPP, "xprod threads must tile the point pairs");
    static constexpr int LS = N + 2;
    static constexpr int NLI = 3 * PX;
    static constexpr long LDS = (2L * 3 * (N / 2 + 1) * PX + CMax<TPLayout<N, NLI, true>::size, NLI * LS>::v + N) *
                                long(2 * sizeof(R));
};

// The schedule compiled as the default for each size: an 8-wide chunk in
// FP32 (a 4-wide one in FP64) keeps the LDS near 52 KB at 256^3 and lets
// three blocks share a CU; from 384^3 on, 4-wide chunks keep two.
template <typename R, int N> struct XDefault {
    static constexpr int TZX0 = (N >= 384) ? 4 : (sizeof(R) == 4 ? 8 : 4);
    static constexpr int TZX = TZX0 < N ? TZX0 : N;
    static constexpr int OCC = N >= 384 ? 2 : 3;
};

template <typename R, int N, int TZX_, int OCC>
__global__ __launch_bounds__(256, OCC) void k_xprod(const typename CplxOf<R>::T* __restrict__ T_all, long t_stride,
                                                  const R* __restrict__ sigma, int a0, int na, R dV, R k_F,
                                                  typename CplxOf<R>::T* __restrict__ Q_all, long q_stride,
                                                  int n_planes, int accumulate, int kx_sup,
                                                  const typename CplxOf<R>::T* __restrict__ tw) {
    using C = typename CplxOf<R>::T;
    using S = Shape<R, N>;
    using X = XShape<R, N, TZX_>;
    constexpr int TZ = X::TZX;
    constexpr int P = X::PX;
    constexpr int NT = X::NTX;
    constexpr int PP = X::PPX;
    constexpr int NZC = N / TZ;
    constexpr int H = N / 2 + 1;
    constexpr long FS = S::FS;
    // line stride of the G / Q lines: N + 2 keeps lanes that store the same
    // x of neighbouring lines (and neighbouring k1 of one line) on distinct banks
    constexpr int LS = N + 2;
    constexpr int NLI = 3 * P;                                   // inverse lines (field, z pair)
    constexpr int NRAW = 3 * H * P;                              // raw pairs per term
    constexpr int TRS = CMax<TPLayout<N, NLI, true>::size, NLI * LS>::v;
    __shared__ __align__(16) C raw[2 * NRAW];                    // [field][kx][pair][2]
    __shared__ C Z[TRS];                                         // transpose, then G lines
    __shared__ C twl[N];
    const int tid = threadIdx.x;
    stage_twiddle_matrix<C, N, TPConst<N>::R1, NT>(twl, tw, tid);   // phase-1 twiddles by (k1, t)
    const int bl = xcd_block(int(blockIdx.x), int(gridDim.x));
    const int zc = bl % NZC;
    const int y = bl / NZC;
    const int z0 = zc * TZ;
    const C* T = T_all + blockIdx.y * t_stride;
    C* Qx = Q_all + blockIdx.y * q_stride;
    C Q[6][PP];
#pragma unroll
    for (int c = 0; c < 6; ++c)
#pragma unroll
        for (int i = 0; i < PP; ++i) Q[c][i] = cmk<C>(R(0), R(0));

    // this block's part of a gradient-field tile (t_offset): one run of TZ
    // z values per kx, TZT apart
    constexpr int TZT = TTile<R, N>::TZT;
    static_assert(TZT % TZ == 0, "an x-pass chunk lies inside one field tile");
    const C* col0 = T + t_offset<N, TZT>(0, y, z0, kx_sup + 1);
    // 16-byte units: a raw element (two complex) is 1 unit in FP32, 2 in FP64
    constexpr int UPE = int(2 * sizeof(C) / 16);
    constexpr int NU = NRAW * UPE;
    constexpr int NIT = (NU + NT - 1) / NT;
    static_assert(NT % 64 == 0 || NT < 64, "global-to-LDS loads are issued per whole wavefront");
    static_assert((3 * FS) * long(sizeof(C)) < (1L << 32), "tile offsets are 32-bit");
    const int lane = tid & 63;
    // byte offset of this lane's unit in each load round, relative to the
    // term's first field: the same for every term; bit i of ld_mask: the
    // unit of round i lies on a plane kx <= kx_sup (else it is zeroed here
    // once and never loaded)
    static_assert(NIT <= 32, "one mask bit per load round");
    unsigned uoff[NIT];
    unsigned ld_mask = 0;
#pragma unroll
    for (int i = 0; i < NIT; ++i) {
        const int u = tid + i * NT;
        const int e = u / UPE, h = u - e * UPE;
        const int j = e / (H * P);
        const int rem = e - j * (H * P);
        const int k = rem / P, p = rem - k * P;
        uoff[i] = unsigned((long(j) * FS + long(k) * TZT + 2 * p) * long(sizeof(C)) + 16 * h);
        if (k <= kx_sup) ld_mask |= 1u << i;
        else if (u < NU) reinterpret_cast<float4*>(raw)[u] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    auto issue_tile = [&](int a, C* dst) {
        const char* colf = reinterpret_cast<const char*>(col0 + long(3 * (a - a0)) * FS);
        char* dstb = reinterpret_cast<char*>(dst);
#pragma unroll
        for (int i = 0; i < NIT; ++i) {
            const int u0 = tid - lane + i * NT;               // uniform in the wavefront
            if (u0 < NU && (i < NIT - 1 || u0 + lane < NU) && ((ld_mask >> i) & 1u)) {
                // lane i of the wavefront lands at dstb + 16 (u0 + i)
                __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)(colf + uoff[i]),
                                                 (__attribute__((address_space(3))) void*)(dstb + 16L * u0), 16, 0,
                                                 0);
            }
        }
    };
    const C* rawc = raw;
    using LayI = TPLayout<N, NLI, true>;
    constexpr int R1 = LayI::R1, R2 = LayI::R2;
    constexpr int ITEMS1 = NLI * R2;
    static_assert(R1 % 2 == 0, "the Hermitian split below assumes an even first radix");
    // phase 1 of the inverse x transform.  Item w -> (j, t, p) with p
    // fastest, then t, then j.  Element n = t + R2 m of inverse line (j, p)
    // packs the z pair (2p, 2p+1) as A + i B, with A, B read at kx = n for
    // m < R1/2 (n < N/2) and conjugated from kx = N - n for m >= R1/2
    // (for n = N/2 both readings agree once the imaginary parts are gone).
    // On the self-conjugate planes kx = 0 and N/2 the imaginary parts are
    // dropped (real-input convention).
    auto phase1 = [&]() {
#pragma unroll
        for (int w0 = 0; w0 < ITEMS1; w0 += NT) {
            const int w = w0 + tid;
            if ((ITEMS1 % NT == 0) || w < ITEMS1) {
                const int p = w % P;
                const int t = (w / P) % R2;
                const int j = w / (P * R2);
                const C* lo = rawc + 2 * ((j * H + t) * P + p);              // kx = t
                const C* hb = rawc + 2 * ((j * H + N / 2 - t) * P + p);      // kx = N/2 - t
                const bool t0 = (t == 0);
                C v[R1];
#pragma unroll
                for (int m = 0; m < R1; ++m) {
                    C a, b;
                    if (m < R1 / 2) {                                        // kx = t + R2 m
                        a = lo[2 * P * R2 * m];
                        b = lo[2 * P * R2 * m + 1];
                    } else {                                                 // kx = N/2 - t - R2 (m - R1/2)
                        a = hb[-2 * P * R2 * (m - R1 / 2)];
                        b = hb[-2 * P * R2 * (m - R1 / 2) + 1];
                    }
                    if ((m == 0 || m == R1 / 2) && t0) {
                        a.y = R(0);
                        b.y = R(0);
                    }
                    v[m] = m < R1 / 2 ? cmk<C>(a.x - b.y, a.y + b.x) : cmk<C>(a.x + b.y, b.x - a.y);
                }
                reg_dft<R1, +1>(v);
#pragma unroll
                for (int k1 = 0; k1 < R1; ++k1) {
                    C o = v[k1];
                    if (k1 > 0) o = cmul(o, tw_at<+1, N>(twl, k1 * R2 + t));
                    Z[LayI::at(j * P + p, k1, t)] = o;
                }
            }
        }
    };

    // Barriers inside a term.  From 384^3 on they hand off LDS only, so the
    // next tile stays in flight through phase 2 and the products (512^3:
    // 15.2-15.5 vs 16.4 ms per launch, 1.6% more HBM reads); up to 256^3 the
    // plain barrier, which lets that tile land by the end of phase 2: the
    // LDS-only form read 6% more from HBM there (the two halves of a tile
    // line, fetched by neighbouring blocks, shared L2 less often) for no
    // gain per launch.
    auto mid_barrier = [] {
        if constexpr (N >= 384) lds_barrier();
        else __syncthreads();
    };
    issue_tile(a0, raw);
    for (int a = a0; a < a0 + na; ++a) {
        __builtin_amdgcn_s_waitcnt(0);    // this wavefront's loads of tile a have landed
        __syncthreads();                  // ... and every wavefront's; Z is free again
        rawc = raw;
        phase1();
        mid_barrier();
        // phase 1 is done with the tile: request the next one.  Phase 1
        // makes no vector memory access (its twiddles come from LDS), since
        // such an access would complete only after every tile load in flight.
        if (a + 1 < a0 + na) issue_tile(a + 1, raw);
        TPRegs<C, N, +1, NLI, NT, true> g;
        g.run(Z, tid);
        mid_barrier();
        g.store([&](int line, int x, C v) { Z[line * LS + x] = v; }, tid);
        mid_barrier();
        const R s = sigma[a] * dV;
#pragma unroll
        for (int i = 0; i < PP; ++i) {
            const int qq = tid + i * NT;
            const int x = qq % N, p = qq / N;
            const C gx = Z[(0 * P + p) * LS + x];
            const C gy = Z[(1 * P + p) * LS + x];
            const C gz = Z[(2 * P + p) * LS + x];
            const C sx = cmk<C>(s * gx.x, s * gx.y);
            const C sy = cmk<C>(s * gy.x, s * gy.y);
            Q[0][i] = cmk<C>(Q[0][i].x + sx.x * gx.x, Q[0][i].y + sx.y * gx.y);
            Q[1][i] = cmk<C>(Q[1][i].x + sy.x * gy.x, Q[1][i].y + sy.y * gy.y);
            Q[2][i] = cmk<C>(Q[2][i].x + s * gz.x * gz.x, Q[2][i].y + s * gz.y * gz.y);
            Q[3][i] = cmk<C>(Q[3][i].x + sx.x * gy.x, Q[3][i].y + sx.y * gy.y);
            Q[4][i] = cmk<C>(Q[4][i].x + sx.x * gz.x, Q[4][i].y + sx.y * gz.y);
            Q[5][i] = cmk<C>(Q[5][i].x + sy.x * gz.x, Q[5][i].y + sy.y * gz.y);
        }
    }
    __syncthreads();
    // forward DFT along x, one component at a time: the P pair lines are
    // staged at Z[0 .. P*LS) and transposed through Z[P*LS ..)
    C* zq = Z;
    C* zt = Z + P * LS;
#pragma unroll
    for (int c = 0; c < 6; ++c) {
#pragma unroll
        for (int i = 0; i < PP; ++i) {
            const int qq = tid + i * NT;
            zq[(qq / N) * LS + (qq % N)] = Q[c][i];
        }
        __syncthreads();
        tp_phase1<C, N, -1, P, NT, false, true>([&](int p, int x) -> C { return zq[p * LS + x]; }, zt, twl, tid);
        __syncthreads();
        TPRegs<C, N, -1, P, NT, false> f;
        f.run(zt, tid);
        f.store([&](int p, int k, C v) { zq[p * LS + k] = v; }, tid);
        __syncthreads();
        for (int e = tid; e < H * P; e += NT) {
            const int k = e / P, p = e % P;
            if (k < n_planes) {
                const C zk = zq[p * LS + k];
                const C zm = zq[p * LS + ((N - k) % N)];
                const C A = cmk<C>(R(0.5) * (zk.x + zm.x), R(0.5) * (zk.y - zm.y));
                const C B = cmk<C>(R(0.5) * (zk.y + zm.y), R(-0.5) * (zk.x - zm.x));
                C* o = Qx + long(c) * FS + (long(k) * N + y) * N + z0 + 2 * p;
                if (accumulate) {
                    const C oa = o[0], ob = o[1];
                    o[0] = cadd(oa, A);
                    o[1] = cadd(ob, B);
                } else {
                    o[0] = A;
                    o[1] = B;
                }
            }
        }
        __syncthreads();
    }
}

// ----------------------------------------------------------------------------
// zbin: last forward pass (z) of the 12 components + TT projection + FP64
// shell sums.  Block = RBB rows (kx, ky); rows that cannot reach the shell
// are skipped.  Q_hat component order per kernel: xx, yy, zz, xy, xz, yz.
// ----------------------------------------------------------------------------
__device__ __forceinline__ double tt_power(const double2* X /* 6 comps */, double kx, double ky, double kz) {
    // Y = P X P with P = 1 - k k^T; returns sum |Y_ij|^2 - |tr Y|^2 / 2.
    const double k[3] = {kx, ky, kz};
    double2 M[3][3];
    M[0][0] = X[0]; M[1][1] = X[1]; M[2][2] = X[2];
    M[0][1] = M[1][0] = X[3];
    M[0][2] = M[2][0] = X[4];
    M[1][2] = M[2][1] = X[5];
    double2 a[3];   // a = X k
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        a[i].x = M[i][0].x * k[0] + M[i][1].x * k[1] + M[i][2].x * k[2];
        a[i].y = M[i][0].y * k[0] + M[i][1].y * k[1] + M[i][2].y * k[2];
    }
    double2 beta;   // k^T X k
    beta.x = k[0] * a[0].x + k[1] * a[1].x + k[2] * a[2].x;
    beta.y = k[0] * a[0].y + k[1] * a[1].y + k[2] * a[2].y;
    double s = 0.0;
    double2 tr;
    tr.x = 0.0;
    tr.y = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            // Y_ij = X_ij - k_i a_j - a_i k_j + beta k_i k_j
            double yr = M[i][j].x - k[i] * a[j].x - a[i].x * k[j] + beta.x * k[i] * k[j];
            double yi = M[i][j].y - k[i] * a[j].y - a[i].y * k[j] + beta.y * k[i] * k[j];
            s += yr * yr + yi * yi;
            if (i == j) {
                tr.x += yr;
                tr.y += yi;
            }
        }
    }
    return s - 0.5 * (tr.x * tr.x + tr.y * tr.y);
}

template <typename R, int N>
__global__ __launch_bounds__(256) void k_zbin(const typename CplxOf<R>::T* __restrict__ Q_all, long q_stride,
                                              const uint8_t* __restrict__ lut_shell, int n2_lo, int n2_hi,
                                              double* __restrict__ part_sum,
                                              unsigned long long* __restrict__ part_cnt,
                                              const typename CplxOf<R>::T* __restrict__ tw) {
    using C = typename CplxOf<R>::T;
    constexpr int RB = Shape<R, N>::RBB_;
    constexpr long FS = Shape<R, N>::FS;
    constexpr int NT = 256;
    constexpr int NL = 12 * RB;
    constexpr int LS = N;
    constexpr int BUF = CMax<TPLayout<N, NL, false>::size, NL * LS>::v;
    __shared__ C buf[BUF];
    __shared__ double rsum[NT / 64];
    __shared__ unsigned long long rcnt[NT / 64];
    const int tid = threadIdx.x;
    const long row0 = long(blockIdx.x) * RB;
    const C* Qxy = Q_all + blockIdx.y * q_stride;
    // can any row of this block reach the shell?
    bool any = false;
    for (int r = 0; r < RB; ++r) {
        const long rr = row0 + r;
        const int kx = int(rr / N), ky = int(rr % N);
        const int nx = signed_index(kx, N), ny = signed_index(ky, N);
        const int mn = nx * nx + ny * ny;
        const int mx = mn + (N / 2) * (N / 2);
        if (mn <= n2_hi && mx >= n2_lo) any = true;
    }
    double acc = 0.0;
    unsigned long long cnt = 0ull;
    if (any) {
        auto ld = [&](int line, int kz) -> C {
            const int comp = line / RB, row = line % RB;
            return Qxy[long(comp) * FS + (row0 + row) * N + kz];
        };
        tp_phase1<C, N, -1, NL, NT, false>(ld, buf, tw, tid);
        __syncthreads();
        TPRegs<C, N, -1, NL, NT, false> f;
        f.run(buf, tid);
        __syncthreads();
        f.store([&](int line, int kz, C v) { buf[line * LS + kz] = v; }, tid);
        __syncthreads();
        for (int e = tid; e < RB * N; e += NT) {
            const int row = e / N, kz = e % N;
            const long rr = row0 + row;
            const int kx = int(rr / N), ky = int(rr % N);
            const int nx = signed_index(kx, N), ny = signed_index(ky, N), nz = signed_index(kz, N);
            const int n2 = nx * nx + ny * ny + nz * nz;
            if (n2 < n2_lo || n2 > n2_hi || !lut_shell[n2]) continue;
            const double inv = 1.0 / sqrt((double)n2);
            const double khx = nx * inv, khy = ny * inv, khz = nz * inv;
            double s = 0.0;
#pragma unroll
            for (int m = 0; m < 2; ++m) {
                double2 X[6];
#pragma unroll
                for (int c = 0; c < 6; ++c) {
                    const C v = buf[((m * 6 + c) * RB + row) * LS + kz];
                    X[c].x = (double)v.x;
                    X[c].y = (double)v.y;
                }
                s += tt_power(X, khx, khy, khz);
            }
            const int w = (kx == 0 || kx == N / 2) ? 1 : 2;
            acc += w * s;
            cnt += (unsigned long long)w;
        }
    }
    // block reduction in a fixed order: wave shuffles, then the waves in order
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        acc += __shfl_down(acc, off, 64);
        cnt += __shfl_down(cnt, off, 64);
    }
    const int lane = tid & 63, wv = tid >> 6;
    if (lane == 0) {
        rsum[wv] = acc;
        rcnt[wv] = cnt;
    }
    __syncthreads();
    if (tid == 0) {
        double t = 0.0;
        unsigned long long c = 0ull;
        for (int i = 0; i < NT / 64; ++i) {
            t += rsum[i];
            c += rcnt[i];
        }
        part_sum[long(blockIdx.y) * gridDim.x + blockIdx.x] = t;
        part_cnt[long(blockIdx.y) * gridDim.x + blockIdx.x] = c;
    }
}

// Lambda(X) = P X P - 1/2 P tr(P X P) of a symmetric X (6 comps xx, yy, zz,
// xy, xz, yz), P = 1 - k k^T: the TT projection whose squared norm tt_power
// returns.
__device__ __forceinline__ void tt_project(const double2* X, double kx, double ky, double kz, double2* Y6) {
    const double k[3] = {kx, ky, kz};
    double2 M[3][3];
    M[0][0] = X[0]; M[1][1] = X[1]; M[2][2] = X[2];
    M[0][1] = M[1][0] = X[3];
    M[0][2] = M[2][0] = X[4];
    M[1][2] = M[2][1] = X[5];
    double2 a[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        a[i].x = M[i][0].x * k[0] + M[i][1].x * k[1] + M[i][2].x * k[2];
        a[i].y = M[i][0].y * k[0] + M[i][1].y * k[1] + M[i][2].y * k[2];
    }
    double2 beta;
    beta.x = k[0] * a[0].x + k[1] * a[1].x + k[2] * a[2].x;
    beta.y = k[0] * a[0].y + k[1] * a[1].y + k[2] * a[2].y;
    double2 Y[3][3];
    double2 tr;
    tr.x = 0.0;
    tr.y = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            Y[i][j].x = M[i][j].x - k[i] * a[j].x - a[i].x * k[j] + beta.x * k[i] * k[j];
            Y[i][j].y = M[i][j].y - k[i] * a[j].y - a[i].y * k[j] + beta.y * k[i] * k[j];
            if (i == j) {
                tr.x += Y[i][j].x;
                tr.y += Y[i][j].y;
            }
        }
    const int ci[6] = {0, 1, 2, 0, 0, 1}, cj[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        const int i = ci[c], j = cj[c];
        const double pij = (i == j ? 1.0 : 0.0) - k[i] * k[j];
        Y6[c].x = Y[i][j].x - 0.5 * pij * tr.x;
        Y6[c].y = Y[i][j].y - 0.5 * pij * tr.y;
    }
}

// Jackknife support: the last forward pass (z) of the 12 components, then
// the TT projection of the shell's modes written back in place (frequency
// space); every other mode is zeroed, including rows that cannot reach the
// shell, so that the inverse transforms that follow see only the shell.
template <typename R, int N>
__global__ __launch_bounds__(256) void k_ztt(typename CplxOf<R>::T* __restrict__ Q, const uint8_t* __restrict__ lut_shell,
                                             int n2_lo, int n2_hi, const typename CplxOf<R>::T* __restrict__ tw) {
    using C = typename CplxOf<R>::T;
    constexpr int RB = Shape<R, N>::RBB_;
    constexpr long FS = Shape<R, N>::FS;
    constexpr int NT = 256;
    constexpr int NL = 12 * RB;
    constexpr int LS = N;
    constexpr int BUF = CMax<TPLayout<N, NL, false>::size, NL * LS>::v;
    __shared__ C buf[BUF];
    const int tid = threadIdx.x;
    const long row0 = long(blockIdx.x) * RB;
    bool any = false;
    for (int r = 0; r < RB; ++r) {
        const long rr = row0 + r;
        const int kx = int(rr / N), ky = int(rr % N);
        const int nx = signed_index(kx, N), ny = signed_index(ky, N);
        const int mn = nx * nx + ny * ny;
        const int mx = mn + (N / 2) * (N / 2);
        if (mn <= n2_hi && mx >= n2_lo) any = true;
    }
    if (!any) {
        for (int e = tid; e < 12 * RB * N; e += NT) {
            const int comp = e / (RB * N), rem = e % (RB * N);
            Q[long(comp) * FS + row0 * N + rem] = cmk<C>(R(0), R(0));
        }
        return;
    }
    auto ld = [&](int line, int kz) -> C {
        const int comp = line / RB, row = line % RB;
        return Q[long(comp) * FS + (row0 + row) * N + kz];
    };
    tp_phase1<C, N, -1, NL, NT, false>(ld, buf, tw, tid);
    __syncthreads();
    TPRegs<C, N, -1, NL, NT, false> f;
    f.run(buf, tid);
    __syncthreads();
    f.store([&](int line, int kz, C v) { buf[line * LS + kz] = v; }, tid);
    __syncthreads();
    for (int e = tid; e < RB * N; e += NT) {
        const int row = e / N, kz = e % N;
        const long rr = row0 + row;
        const int kx = int(rr / N), ky = int(rr % N);
        const int nx = signed_index(kx, N), ny = signed_index(ky, N), nz = signed_index(kz, N);
        const int n2 = nx * nx + ny * ny + nz * nz;
        const bool in = n2 >= n2_lo && n2 <= n2_hi && lut_shell[n2];
        const double inv = in ? 1.0 / sqrt((double)n2) : 0.0;
#pragma unroll
        for (int m = 0; m < 2; ++m) {
            double2 X[6], Y[6];
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                const C v = buf[((m * 6 + c) * RB + row) * LS + kz];
                X[c].x = (double)v.x;
                X[c].y = (double)v.y;
            }
            tt_project(X, nx * inv, ny * inv, nz * inv, Y);
#pragma unroll
            for (int c = 0; c < 6; ++c)
                Q[long(m * 6 + c) * FS + rr * N + kz] = in ? cmk<C>((R)Y[c].x, (R)Y[c].y) : cmk<C>(R(0), R(0));
        }
    }
}

// E[x] = (first ? 0 : E[x]) + w h[x]^2, in FP64
template <typename R>
__global__ __launch_bounds__(256) void k_energy_accum(const R* __restrict__ h, double* __restrict__ E, long total,
                                                      double w, int first) {
    const long i = long(blockIdx.x) * 256 + threadIdx.x;
    if (i >= total) return;
    const double v = (double)h[i];
    E[i] = (first ? 0.0 : E[i]) + w * v * v;
}

// out[(a M + b) M + c] = sum of E over the sub-volume x in [a, a+1) N/M,
// y in [b, b+1) N/M, z in [c, c+1) N/M; one block per sub-volume, fixed-order
// reduction.
__global__ __launch_bounds__(256) void k_subvol_sums(const double* __restrict__ E, int N, int M,
                                                     double* __restrict__ out) {
    __shared__ double red[256];
    const int sv = blockIdx.x;
    const int a = sv / (M * M), b = (sv / M) % M, c = sv % M;
    const int B = N / M;
    const long nsite = long(B) * B * B;
    double acc = 0.0;
    for (long t = threadIdx.x; t < nsite; t += 256) {
        const int z = int(t % B), y = int((t / B) % B), x = int(t / (long(B) * B));
        acc += E[(long(a * B + x) * N + (b * B + y)) * N + (c * B + z)];
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[sv] = red[0];
}

__global__ __launch_bounds__(256) void k_finalize(const double* __restrict__ ps_all,
                                                  const unsigned long long* __restrict__ pc_all, int n,
                                                  double* __restrict__ out_sum, unsigned long long* __restrict__ out_cnt,
                                                  int out_stride) {
    __shared__ double rs[256];
    __shared__ unsigned long long rc[256];
    const int tid = threadIdx.x;
    const double* ps = ps_all + long(blockIdx.x) * n;
    const unsigned long long* pc = pc_all + long(blockIdx.x) * n;
    double a = 0.0;
    unsigned long long c = 0ull;
    for (int i = tid; i < n; i += 256) {
        a += ps[i];
        c += pc[i];
    }
    rs[tid] = a;
    rc[tid] = c;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) {
            rs[tid] += rs[tid + s];
            rc[tid] += rc[tid + s];
        }
        __syncthreads();
    }
    if (tid == 0) {
        out_sum[long(blockIdx.x) * out_stride] = rs[0];
        out_cnt[long(blockIdx.x) * out_stride] = rc[0];
    }
}

// ----------------------------------------------------------------------------
// Engine specialisation
// ----------------------------------------------------------------------------
template <typename R, int NN> struct EngineImpl final : Engine {
    using C = typename CplxOf<R>::T;
    using S = Shape<R, NN>;
    const C* tw;
    explicit EngineImpl(const void* twd) : tw(static_cast<const C*>(twd)) { add_schedules(); }

    int N() const override { return NN; }
    size_t real_bytes() const override { return sizeof(R); }
    size_t complex_bytes() const override { return sizeof(C); }
    int zbin_blocks() const override { return int((long(S::H) * NN) / S::RBB_); }
    int sumsq_blocks() const override { return 1024; }

    void noise(uint64_t seed, void* out, hipStream_t s) override {
        const long total = long(NN) * NN * NN;
        k_noise<R><<<dim3(unsigned((total + 255) / 256)), dim3(256), 0, s>>>(static_cast<R*>(out), total, seed);
    }
    void xpass_r2c(const void* in, void* out, hipStream_t s) override {
        k_xpass_r2c<R, NN><<<dim3(NN * (NN / S::TZ)), dim3(XCfg<R, NN>::NT), 0, s>>>(static_cast<const R*>(in),
                                                                      static_cast<C*>(out), tw);
    }
    void xpass_c2r(const void* in, void* out, hipStream_t s) override {
        k_xpass_c2r<R, NN><<<dim3(NN * (NN / S::TZ)), dim3(XCfg<R, NN>::NT), 0, s>>>(static_cast<const C*>(in),
                                                                      static_cast<R*>(out), tw);
    }
    void ypass(void* data, int n_fields, long field_stride, int n_planes, int sign, int nb, long batch_stride,
               hipStream_t s) override {
        const unsigned blocks = unsigned(long(n_fields) * n_planes * (NN / S::TZ));
        if (blocks == 0 || nb <= 0) return;
        const dim3 grid(blocks, unsigned(nb));
        if (sign < 0)
            k_ypass<R, NN, -1><<<grid, dim3(YCfg<R, NN>::NT), 0, s>>>(static_cast<C*>(data), field_stride, n_planes,
                                                                      batch_stride, tw);
        else
            k_ypass<R, NN, +1><<<grid, dim3(YCfg<R, NN>::NT), 0, s>>>(static_cast<C*>(data), field_stride, n_planes,
                                                                      batch_stride, tw);
    }
    void zpass(void* data, long n_rows, int sign, hipStream_t s) override {
        const unsigned blocks = unsigned((n_rows + ZCfg<R, NN>::RB - 1) / ZCfg<R, NN>::RB);
        if (blocks == 0) return;
        if (sign < 0)
            k_zpass<R, NN, -1><<<dim3(blocks), dim3(256), 0, s>>>(static_cast<C*>(data), n_rows, tw);
        else
            k_zpass<R, NN, +1><<<dim3(blocks), dim3(256), 0, s>>>(static_cast<C*>(data), n_rows, tw);
    }
    void filter(void* half, const double* amp, hipStream_t s) override {
        k_filter<R, NN><<<dim3(unsigned((S::FS + 255) / 256)), dim3(256), 0, s>>>(static_cast<C*>(half), amp);
    }
    void laplacian(void* half, double c, hipStream_t s) override {
        k_laplacian<R, NN><<<dim3(unsigned((S::FS + 255) / 256)), dim3(256), 0, s>>>(static_cast<C*>(half), c);
    }
    void square(const void* in, void* out, hipStream_t s) override {
        const long total = long(NN) * NN * NN;
        k_square<R><<<dim3(unsigned((total + 255) / 256)), dim3(256), 0, s>>>(static_cast<const R*>(in),
                                                                           static_cast<R*>(out), total);
    }
    void nonlocal_combine(const void* zg, const void* l1, const void* l2, void* out, hipStream_t s) override {
        const long total = long(NN) * NN * NN;
        k_nonlocal_combine<R><<<dim3(unsigned((total + 255) / 256)), dim3(256), 0, s>>>(
            static_cast<const R*>(zg), static_cast<const R*>(l1), static_cast<const R*>(l2), static_cast<R*>(out),
            total);
    }
    void sumsq(const void* real, double* partials, double* out, hipStream_t s) override {
        const long total = long(NN) * NN * NN;
        k_sumsq_partial<R><<<dim3(1024), dim3(256), 0, s>>>(static_cast<const R*>(real), total, partials);
        k_reduce_sum<<<dim3(1), dim3(256), 0, s>>>(partials, 1024, out);
    }
    void map_scale(const void* in, void* out, const double* sum_sq, const MapParams& mp, double scale,
                   hipStream_t s) override {
        const long total = long(NN) * NN * NN;
        k_map_scale<R><<<dim3(unsigned((total + 255) / 256)), dim3(256), 0, s>>>(
            static_cast<const R*>(in), static_cast<R*>(out), total, sum_sq, mp, scale);
    }
    void restrict_half(const void* src, int n_src, const int* sel, int nb, void* dst, hipStream_t s) override {
        if (nb <= 0 || n_src <= NN) return;
        k_restrict<R, NN><<<dim3(unsigned((S::FS + 255) / 256), unsigned(nb)), dim3(256), 0, s>>>(
            static_cast<const C*>(src), n_src, sel, static_cast<C*>(dst));
    }
    void lut(double k_F, double k_target, double k_lo, double k_hi, const double* edges, int n_modes,
             int16_t* lut_u, uint8_t* lut_shell, hipStream_t s) override {
        const int n2max = S::N2MAX;
        k_lut<<<dim3(unsigned(n2max / 256 + 1)), dim3(256), 0, s>>>(n2max, k_F, k_target, k_lo, k_hi, edges,
                                                                    n_modes, lut_u, lut_shell);
    }
    // highest kx plane inside the support bound: min(N/2, floor(sqrt(n2_sup)))
    static int kx_sup_of(int n2_sup) {
        long r = long(std::sqrt(double(n2_sup)));
        while ((r + 1) * (r + 1) <= n2_sup) ++r;
        while (r > 0 && r * r > n2_sup) --r;
        return int(std::min<long>(r, NN / 2));
    }
    void gen_z(const void* phi_hat, const int* sel, int nb, const int16_t* lut_u, const void* phi_tab, int n_alpha,
               int a0, int na, double k_F, double inv_V, void* Sd, long s_stride, int n2_sup,
               hipStream_t s) override {
        constexpr int RB = GCfg<R, NN>::RB;
        if (nb <= 0 || na <= 0 || n2_sup < 0) return;
        const int kxs = kx_sup_of(n2_sup);
        const int c0 = live_row_blocks<NN, RB>(ylim_of<NN>(n2_sup));
        const int nrb = (kxs + 1) * c0;
        long live = 0;                                       // live row blocks of all planes
        for (int kx = 0; kx <= kxs; ++kx) live += live_row_blocks<NN, RB>(ylim_of<NN>(n2_sup - kx * kx));
        // about 4096 busy blocks per launch (16 per CU) when the support allows
        constexpr long kBusy = 4096;
        const long want = (kBusy + live * nb - 1) / std::max(1L, live * nb);
        const int ng0 = int(std::min<long>(std::max<long>(want, 1), na));
        const int tg = (na + ng0 - 1) / ng0;
        const int ng = (na + tg - 1) / tg;
        k_gen_z<R, NN><<<dim3(unsigned(long(nrb) * ng), unsigned(nb)), dim3(GCfg<R, NN>::NT), 0, s>>>(
            static_cast<const C*>(phi_hat), sel, lut_u, static_cast<const R*>(phi_tab), n_alpha, a0, na, R(k_F),
            R(inv_V), static_cast<C*>(Sd), s_stride, n2_sup, c0, nrb, tg, tw);
    }
    void ypass3(const void* Sd, int na, int nb, long s_stride, void* T, long t_stride, double k_F, int n2_sup,
                hipStream_t s) override {
        const int hs = kx_sup_of(n2_sup) + 1;
        const unsigned blocks = unsigned(long(na) * hs * (NN / YCfg<R, NN>::TZ));
        if (blocks == 0 || nb <= 0 || n2_sup < 0) return;
        k_ypass3<R, NN><<<dim3(blocks, unsigned(nb)), dim3(YCfg<R, NN>::NT), 0, s>>>(
            static_cast<const C*>(Sd), s_stride, static_cast<C*>(T), t_stride, R(k_F), n2_sup, hs, tw);
    }
    void xprod(const void* T, long t_stride, int nb, const void* sigma_tab, int a0, int na, double dV, double k_F,
               void* Qx, long q_stride, int n_planes, int accumulate, int kx_sup, hipStream_t s) override {
        xs_[xsel_].fn(static_cast<const C*>(T), t_stride, nb, static_cast<const R*>(sigma_tab), a0, na, R(dV),
                      R(k_F), static_cast<C*>(Qx), q_stride, n_planes, accumulate, std::min(kx_sup, NN / 2), tw, s);
    }
    int xprod_schedules() const override { return nxs_; }
    void xprod_schedule_info(int i, int* tzx, int* occ) const override {
        *tzx = xs_[i].tzx;
        *occ = xs_[i].occ;
    }
    void set_xprod_schedule(int i) override { xsel_ = i; }
    int xprod_schedule() const override { return xsel_; }

    // x-pass schedules compiled for this size: entry 0 is the default, the
    // others differ in chunk width (half, double) and blocks-per-CU target.
    using XFn = void (*)(const C*, long, int, const R*, int, int, R, R, C*, long, int, int, int, const C*,
                         hipStream_t);
    struct XSched {
        int tzx, occ;
        XFn fn;
    };
    XSched xs_[3];
    int nxs_ = 0, xsel_ = 0;
    template <int TZX, int OCC>
    static void xlaunch(const C* T, long t_stride, int nb, const R* sigma, int a0, int na, R dV, R kF, C* Qx,
                        long q_stride, int n_planes, int acc, int kx_sup, const C* twd, hipStream_t s) {
        using X = XShape<R, NN, TZX>;
        const unsigned blocks = unsigned(NN * (NN / X::TZX));
        k_xprod<R, NN, TZX, OCC><<<dim3(blocks, unsigned(nb)), dim3(X::NTX), 0, s>>>(
            T, t_stride, sigma, a0, na, dV, kF, Qx, q_stride, n_planes, acc, kx_sup, twd);
    }
    template <int TZX, int OCC> void add_schedule() {
        using X = XShape<R, NN, TZX>;
        if constexpr (TZX >= 2 && TZX <= NN && TTile<R, NN>::TZT % TZX == 0 && X::LDS <= 160 * 1024)
            xs_[nxs_++] = {X::TZX, OCC, &xlaunch<TZX, OCC>};
    }
    void add_schedules() {
        using D = XDefault<R, NN>;
        add_schedule<D::TZX, D::OCC>();
        if constexpr (NN >= 64) {
            add_schedule<D::TZX / 2, D::OCC>();
            add_schedule<D::TZX * 2, (D::OCC > 1 ? D::OCC - 1 : 1)>();
        }
    }
    void zbin(const void* Qxy, int nb, long q_stride, const uint8_t* lut_shell, int n2_lo, int n2_hi, double* ps,
              unsigned long long* pc, hipStream_t s) override {
        k_zbin<R, NN><<<dim3(unsigned(zbin_blocks()), unsigned(nb)), dim3(256), 0, s>>>(
            static_cast<const C*>(Qxy), q_stride, lut_shell, n2_lo, n2_hi, ps, pc, tw);
    }
    void ztt(void* Q, const uint8_t* lut_shell, int n2_lo, int n2_hi, hipStream_t s) override {
        k_ztt<R, NN><<<dim3(unsigned(zbin_blocks())), dim3(256), 0, s>>>(static_cast<C*>(Q), lut_shell, n2_lo, n2_hi,
                                                                         tw);
    }
    void energy_accum(const void* h, double* E, double w, int first, hipStream_t s) override {
        const long total = long(NN) * NN * NN;
        k_energy_accum<R><<<dim3(unsigned((total + 255) / 256)), dim3(256), 0, s>>>(static_cast<const R*>(h), E,
                                                                                   total, w, first);
    }
    void subvol_sums(const double* E, int M, double* out, hipStream_t s) override {
        k_subvol_sums<<<dim3(unsigned(M * M * M)), dim3(256), 0, s>>>(E, NN, M, out);
    }
    void finalize(const double* ps, const unsigned long long* pc, int n, int nb, double* out_sum,
                  unsigned long long* out_cnt, int out_stride, hipStream_t s) override {
        k_finalize<<<dim3(unsigned(nb)), dim3(256), 0, s>>>(ps, pc, n, out_sum, out_cnt, out_stride);
    }
};

template <typename R> static Engine* make_for(int N, const void* tw) {
    switch (N) {
        case 8: return new EngineImpl<R, 8>(tw);
        case 16: return new EngineImpl<R, 16>(tw);
        case 32: return new EngineImpl<R, 32>(tw);
        case 64: return new EngineImpl<R, 64>(tw);
        case 128: return new EngineImpl<R, 128>(tw);
        case 256: return new EngineImpl<R, 256>(tw);
        case 384: return new EngineImpl<R, 384>(tw);
        case 512: return new EngineImpl<R, 512>(tw);
        default: return nullptr;
    }
}

Engine* make_engine(int prec, int N, const void* tw) {
    return prec == 1 ? make_for<double>(N, tw) : make_for<float>(N, tw);
}

void host_twiddles(int prec, int N, void* out) {
    for (int t = 0; t < N; ++t) {
        // exp(-2 pi i t / N) from an exactly reduced angle
        const long double a = -2.0L * 3.14159265358979323846264338327950288L * (long double)t / (long double)N;
        const long double c = cosl(a), s = sinl(a);
        if (prec == 1) {
            static_cast<double*>(out)[2 * t] = (double)c;
            static_cast<double*>(out)[2 * t + 1] = (double)s;
        } else {
            static_cast<float*>(out)[2 * t] = (float)c;
            static_cast<float*>(out)[2 * t + 1] = (float)s;
        }
    }
}

}  // namespace sigw
