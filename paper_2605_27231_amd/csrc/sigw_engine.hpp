// Interface between the host-side plan (sigw_plan.cpp) and the templated
// device kernels (sigw_kernels.hip).  One Engine instance exists per plan,
// specialised for the plan's precision and lattice size; each method enqueues
// exactly one kernel launch (so that it can be timed on its own) unless noted.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace sigw {

struct MapParams {
    int kind;          // 0 Gaussian, 1 local, 2 exponential tail
    double F_NL, G_NL, beta, clip;
};

struct Engine {
    virtual ~Engine() = default;
    virtual int N() const = 0;
    virtual size_t real_bytes() const = 0;      // sizeof of the path real type
    virtual size_t complex_bytes() const = 0;   // sizeof of the path complex type
    virtual int zbin_blocks() const = 0;         // partial sums produced by zbin
    virtual int sumsq_blocks() const = 0;

    // Philox white noise, one deviate per site (real layout).
    virtual void noise(uint64_t seed, void* real_out, hipStream_t s) = 0;
    // Forward DFT along x of a real field into the half layout.
    virtual void xpass_r2c(const void* real_in, void* half_out, hipStream_t s) = 0;
    // Inverse DFT along x of a half spectrum into a real field.
    virtual void xpass_c2r(const void* half_in, void* real_out, hipStream_t s) = 0;
    // Complex DFT along y, in place, of n_fields half spectra spaced by
    // field_stride complex elements, on the kx planes [0, n_planes), for nb
    // batch members spaced by batch_stride.
    virtual void ypass(void* data, int n_fields, long field_stride, int n_planes, int sign, int nb,
                       long batch_stride, hipStream_t s) = 0;
    // Complex DFT along z, in place, of n_rows contiguous rows.
    virtual void zpass(void* data, long n_rows, int sign, hipStream_t s) = 0;
    // Multiply a half spectrum by amp[|n|^2] (FP64 table, rounded to the path precision).
    virtual void filter(void* half, const double* amp_by_n2, hipStream_t s) = 0;
    // out[0] = sum_x X(x)^2 in FP64 (two launches: block partials, fixed-order total).
    virtual void sumsq(const void* real, double* partials, double* out, hipStream_t s) = 0;
    // real_out = scale * map(real_in), evaluated in FP64; m2 = <zeta_g^2> on the device.
    virtual void map_scale(const void* real_in, void* real_out, const double* sum_sq,
                           const MapParams& mp, double scale, hipStream_t s) = 0;
    // Non-local map pieces: half *= c |n|^2 (spectral Laplacian with c =
    // -k_F^2 times any coefficient and normalisation, evaluated in FP64);
    // out = in^2; out = zg + l1 + zg l2 (FP64 per site).
    virtual void laplacian(void* half, double c, hipStream_t s) = 0;
    virtual void square(const void* in, void* out, hipStream_t s) = 0;
    virtual void nonlocal_combine(const void* zg, const void* l1, const void* l2, void* out, hipStream_t s) = 0;
    // Half spectrum of this (smaller) grid taken from half spectra of an
    // n_src grid: dst[b] gets slot sel[b] of src at every mode of this grid
    // (signed indices |n_y|, |n_z| <= N/2, the index -N/2 read at n = -N/2 of
    // the source).  Exact copies; the caller ensures the field it serves has
    // no support outside |n_c| < N/2.
    virtual void restrict_half(const void* src, int n_src, const int* sel, int nb, void* dst,
                               hipStream_t s) = 0;
    // Per-target tables over integer |n|^2 in [0, 3 (N/2)^2]: u-interval index
    // of u = k_F sqrt(n2) / k_target (-1 outside) and shell membership
    // k_lo <= k_F sqrt(n2) < k_hi, n2 > 0.
    virtual void lut(double k_F, double k_target, double k_lo, double k_hi, const double* edges,
                     int n_modes, int16_t* lut_u, uint8_t* lut_shell, hipStream_t s) = 0;
    // Every per-target kernel below runs nb batch members in one launch
    // (grid y); member b works on the realisation in slot sel[b] and on its
    // own workspace, found at b times the given stride.
    //
    // Support bound n2_sup: every mode with phi_a(u(n)) != 0 has |n|^2 <=
    // n2_sup.  A (kx, ky) row with nx^2 + ny^2 > n2_sup is zero after the z
    // pass and a kx plane with kx^2 > n2_sup is zero after the y pass; gen_z
    // does not write such rows, ypass3 reads them as zeros and writes only
    // the planes kx <= kx_sup = min(N/2, floor(sqrt(n2_sup))), and xprod
    // reads only those planes.  All three must get the same bound.
    //
    // Fused weighting + inverse DFT along z: for a = a0..a0+na-1,
    // S[2(a-a0)] = IDFT_z( phi_a(u) Phi_hat / V ), S[2(a-a0)+1] = IDFT_z( i qt_z phi_a(u) Phi_hat / V ).
    virtual void gen_z(const void* phi_hat_slots, const int* sel, int nb, const int16_t* lut_u,
                       const void* phi_tab, int n_alpha, int a0, int na, double k_F, double inv_V,
                       void* S, long s_stride, int n2_sup, hipStream_t s) = 0;
    // Inverse DFT along y of na terms' (W, Z) pairs into their three gradient
    // fields T[3a + j]: i qt_x IDFT_y(W), IDFT_y(i qt_y W), IDFT_y(Z), stored
    // in the x-pass tile layout.
    virtual void ypass3(const void* S, int na, int nb, long s_stride, void* T, long t_stride, double k_F,
                        int n2_sup, hipStream_t s) = 0;
    // Fused inverse DFT along x + products + forward DFT along x:
    // Qx_c = DFT_x( sum_a sigma_a dV G_a,i G_a,j ) for the 6 components, on
    // the kx planes [0, n_planes); accumulate adds into Qx instead of storing.
    // The planes kx > kx_sup of T are taken as zero and not read.
    // Runs the active x-pass schedule.
    virtual void xprod(const void* T, long t_stride, int nb, const void* sigma_tab, int a0, int na,
                       double dV, double k_F, void* Qx, long q_stride, int n_planes, int accumulate,
                       int kx_sup, hipStream_t s) = 0;
    // x-pass schedules compiled for this size (index 0 is the default): z
    // chunk width and blocks-per-CU target of schedule i; the active one.
    // Every schedule computes the same values in the same order.
    virtual int xprod_schedules() const = 0;
    virtual void xprod_schedule_info(int i, int* tzx, int* occ) const = 0;
    virtual void set_xprod_schedule(int i) = 0;
    virtual int xprod_schedule() const = 0;
    // Fused forward DFT along z of the 12 components (both kernels) + TT
    // projection + shell sums: one (sum, count) partial per block, member b's
    // at [b * zbin_blocks(), (b + 1) * zbin_blocks()).
    virtual void zbin(const void* Qxy, int nb, long q_stride, const uint8_t* lut_shell, int n2_lo,
                      int n2_hi, double* partial_sum, unsigned long long* partial_cnt,
                      hipStream_t s) = 0;
    // Jackknife support (one realisation): forward z pass of the 12
    // components + TT projection of the shell's modes written back in place,
    // everything else zeroed; E = (first ? 0 : E) + w h^2 per site in FP64;
    // the sums of E over the M^3 sub-volumes.
    virtual void ztt(void* Q, const uint8_t* lut_shell, int n2_lo, int n2_hi, hipStream_t s) = 0;
    virtual void energy_accum(const void* h, double* E, double w, int first, hipStream_t s) = 0;
    virtual void subvol_sums(const double* E, int M, double* out, hipStream_t s) = 0;
    // Fixed-order reduction of each member's n partials into
    // out_sum[b * out_stride], out_cnt[b * out_stride].
    virtual void finalize(const double* partial_sum, const unsigned long long* partial_cnt, int n, int nb,
                          double* out_sum, unsigned long long* out_cnt, int out_stride,
                          hipStream_t s) = 0;
};

// Returns nullptr for an unsupported (prec, N).
Engine* make_engine(int prec, int N, const void* twiddles_dev);
// Host twiddles exp(-2 pi i t / N), t = 0..N-1, in the path precision (interleaved).
void host_twiddles(int prec, int N, void* out);

}  // namespace sigw
