/*
 * sigw.h -- C ABI of the MI355X (gfx950) library that computes the
 * scalar-induced gravitational-wave spectrum Omega^(RD)_GW(k) of a (non-)
 * Gaussian curvature field on a 3D periodic lattice, by the separable-kernel
 * convolution method of arXiv 2605.27231 (Piccoli).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Lattice: N sites per side (even), box side L, k_F = 2 pi / L, cell volume
 *   dV = (L/N)^3, volume V = L^3.  Modes n are integer triples with signed
 *   representatives in [-N/2, N/2); q = k_F n.
 * Fourier convention (Sec. III two-point function, Sec. IV real-space fields):
 *   X_hat(n) = dV sum_x exp(-i q.x) X(x),  X(x) = (1/V) sum_n exp(i q.x) X_hat(n).
 * Layouts (row-major, last index fastest, no padding):
 *   real field      [x][y][z], N*N*N elements of the path precision;
 *   half spectrum   [kx][ky][kz] with kx = 0..N/2 (the first axis is halved;
 *                   kx = N/2 is the Nyquist plane), ky, kz = 0..N-1;
 *                   (N/2+1)*N*N complex elements, interleaved (re, im) of the
 *                   path precision.  It equals numpy.fft.fftn(X)[:N//2+1] * dV.
 * Precision: SIGW_F32 runs fields and FFTs in float/complex64, SIGW_F64 in
 *   double/complex128.  Shell sums, the <zeta_g^2> reduction, the maps and all
 *   lookup tables are FP64 in both.
 * Streams: a plan enqueues all device work on the HIP stream given at
 *   creation (NULL = the null stream).  Entry points that return host results
 *   synchronise that stream; the others only enqueue.
 * Memory: device pointers are borrowed for the duration of the call (the work
 *   they feed is enqueued on the plan stream, so the caller keeps them alive
 *   until that stream reaches the call); host pointers are read or written
 *   before the call returns.  The plan owns every buffer it allocates and
 *   frees them in sigw_plan_destroy.
 * Errors: no exception crosses the ABI.  Invalid arguments return
 *   SIGW_E_INVALID and change nothing; a HIP failure returns SIGW_E_DEVICE;
 *   a call out of order (e.g. a spectrum before any field) returns
 *   SIGW_E_STATE.  sigw_last_error(plan) gives a text for the last failure.
 * Threads: a plan is used by one host thread at a time; distinct plans are
 *   independent and may run concurrently on different streams.
 */
#ifndef SIGW_H
#define SIGW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sigw_plan* sigw_plan_t;

typedef enum {
    SIGW_OK = 0,
    SIGW_E_INVALID = -1,
    SIGW_E_NOMEM = -2,
    SIGW_E_DEVICE = -3,
    SIGW_E_UNSUPPORTED = -4,
    SIGW_E_STATE = -5,
    SIGW_E_PENDING = -6
} sigw_status;

typedef enum { SIGW_F32 = 0, SIGW_F64 = 1 } sigw_prec;

typedef enum { SIGW_MAP_GAUSS = 0, SIGW_MAP_LOCAL = 1, SIGW_MAP_EXPTAIL = 2, SIGW_MAP_NONLOCAL = 3 } sigw_map_kind;

/* Plan description: the lattice and the separable decomposition of Sec. V.
 * N must be one of 8, 16, 32, 64, 128, 256, 384, 512 (2^a 3^b sizes with a
 * compiled FFT schedule).  n_modes intervals on [u_min, u_max) with the grid
 * density rho(u) = 1 + A_p exp(-(u-u_p)^2 / (2 sigma_p^2)) (Eq. grid_density);
 * 1 <= n_alpha <= n_modes terms are kept (Eq. decomposition).
 * n_slots is the number of device-resident Phi_hat fields (realisations) the
 * plan holds, >= 1.  alpha_chunk bounds how many separable terms share one
 * workspace pass (0 = all n_alpha; a smaller value trades a few extra
 * read-modify-write passes for 3*alpha_chunk instead of 3*n_alpha fields of
 * workspace).  scratch_terms is how many terms the first inverse pass
 * stages at a time (2 half spectra each) before they are expanded into
 * their gradient fields; 0 picks the largest count (up to alpha_chunk) whose
 * staging fits in 16 GiB.  A small count keeps the staging resident in the
 * last-level cache at the price of re-reading Phi_hat per group.  batch is
 * how many realisations one kernel launch processes together (0 = 1); each
 * brings its own workspace, so the footprint grows linearly with it.
 * autotune: 0 = the compiled default x-pass schedule; 1 = at creation, the
 * schedule the process-wide table holds for this (device, N, precision), or
 * if there is none, run sigw_autotune (see below). */
typedef struct {
    int32_t N;
    double  L;
    int32_t prec;        /* sigw_prec */
    int32_t n_slots;
    int32_t n_modes;
    int32_t n_alpha;
    double  u_min, u_max, u_p, sigma_p, A_p;
    int32_t alpha_chunk;
    int32_t scratch_terms;
    int32_t batch;
    int32_t autotune;
} sigw_plan_desc;

/* Log-normal peak, Eq. lognormal: Delta^2(k) = A/sqrt(2 pi sigma^2) exp(-ln^2(k/k_star)/(2 sigma^2)).
 * The field's spectrum is P(k) = 2 pi^2 Delta^2(k) / k^3.  A >= 0, sigma > 0, k_star > 0. */
typedef struct { double A, sigma, k_star; } sigw_lognormal;

/* Non-Gaussian map (Sec. VI B, Sec. VI C and the exponential-tail family):
 *   GAUSS:    zeta = zeta_g
 *   LOCAL:    zeta = zeta_g + F_NL (zeta_g^2 - <zeta_g^2>) + G_NL zeta_g^3,
 *             <zeta_g^2> the FP64 mean over the lattice
 *   EXPTAIL:  zeta = -ln(max(1 - beta zeta_g, clip)) / beta, beta > 0, clip > 0
 *   NONLOCAL: zeta = zeta_g + (alpha_NL / k_NL^2) lap(zeta_g^2)
 *                    + (beta_NL / k_NL^2) zeta_g lap(zeta_g)      (Eq. nonlocal)
 *             with the spectral Laplacian lap X = IDFT(-|k_F n|^2 DFT X) (the
 *             Nyquist index keeps its value); k_NL > 0 is the peak scale.
 *             Uses the plan's gradient-field workspace as scratch. */
typedef struct { int32_t kind; double F_NL, G_NL, beta, clip, alpha_NL, beta_NL, k_NL; } sigw_ngmap;

/* Fill d with the paper's default decomposition (n_modes 200, n_alpha 50,
 * u in [1e-3, 15), u_p 1, sigma_p 0.5, A_p 10), one slot, all terms per
 * pass, automatic staging. */
sigw_status sigw_plan_desc_default(sigw_plan_desc* d, int32_t N, double L, int32_t prec);

/* Device bytes a plan with this description allocates (for admission by HBM
 * budget).  Host only; no device is touched. */
sigw_status sigw_plan_footprint(const sigw_plan_desc* d, size_t* bytes);

/* Build a plan: validate, build the kernel tables on the host (Sec. V:
 * u-grid, C_ij = sqrt(L_i L_j) I(c_i, c_j) on the triangle strip, symmetric
 * eigen-decomposition, keep n_alpha terms by |sigma|), upload them, build the
 * FFT twiddles and allocate the workspace.  hip_stream is a hipStream_t or
 * NULL.  On success *out owns everything it allocated. */
sigw_status sigw_plan_create(const sigw_plan_desc* d, void* hip_stream, sigw_plan_t* out);
sigw_status sigw_plan_destroy(sigw_plan_t plan);

/* Host-only copy of the kernel table the plan would use for kernel m
 * (0 = I_s, 1 = I_c, Eq. kernels): sigma[n_alpha] (ordered by |sigma|
 * descending), phi[n_modes * n_alpha] (phi_a on interval i at
 * phi[i * n_alpha + a]), edges[n_modes + 1].  Any output may be NULL. */
sigw_status sigw_kernel_table(const sigw_plan_desc* d, int32_t m, double* sigma, double* phi,
                              double* edges);

/* Host-only table of the same layout for a background of constant equation
 * of state w, 0 < w < 1, with adiabatic pressure (c_s^2 = w): the kernels
 * I_m^w(u, v) are the asymptotic envelope time integrals of Sec. IV with
 * Sec. II's ingredients for that background (Eq. scalar and the homogeneous
 * wave equation solved by Bessel functions, the Wronskian from Abel's
 * identity, the 2/(3(1+w)) source factor), including the factor
 * [3(1+w)/(5+3w) / (2/3)]^2 that converts the initial potential of Sec. II
 * to the Phi = 2 zeta / 3 the lattice path carries.  At w = 1/3 they are
 * Eq. kernels.  Decomposed on the grid of d as in Sec. V; install with
 * sigw_plan_set_kernel_table (both m).  The Omega normalisation of Sec. III
 * is the radiation-era one; for w != 1/3 the spectrum returned is that
 * expression evaluated with these envelopes.  Takes seconds the first time
 * for each (grid, w) in the process (cached).  SIGW_E_INVALID for m not in
 * {0, 1}, w outside (0, 1), or sqrt(w) u_min below ~1e-3. */
sigw_status sigw_kernel_table_w(const sigw_plan_desc* d, double w, int32_t m, double* sigma, double* phi,
                                double* edges);

/* Replace kernel m's separable table in a plan with the caller's own, in the
 * layout sigw_kernel_table returns: sigma[n_alpha], phi[n_modes * n_alpha]
 * (phi_a on interval i at phi[i * n_alpha + a]) and, unless NULL, the u grid
 * edges[n_modes + 1], which both kernels share (a new grid replaces it for
 * m = 0 and 1 alike, so set both tables on it).  n_modes and n_alpha are
 * the plan's.  The sum_a sigma_a phi_a(u) phi_a(v) then stands for the
 * kernel I_m(u, v) of Eq. decomposition whatever it was built from: tables
 * for other equations of state or thermal histories, other grids or bases
 * (the device path reads only the table).  phi_a is zero outside
 * [edges[0], edges[n_modes]).  Host arrays, read during the call; waits for
 * the plan's enqueued work, then copies.  Spectrum graphs of the plan
 * (sigw_graph_create) read the new tables when launched; a graph captured
 * before a new u grid was set keeps the support bounds and grids of the old
 * one, so sigw_graph_launch refuses it with SIGW_E_STATE: create it again.  SIGW_E_INVALID for m not in
 * {0, 1}, NULL sigma or phi, non-finite values, or edges not strictly
 * increasing from a value >= 0; the plan is then unchanged. */
sigw_status sigw_plan_set_kernel_table(sigw_plan_t plan, int32_t m, const double* sigma, const double* phi,
                                       const double* edges);

/* White noise of one seed: one N(0,1) deviate per site (Philox4x64-10 with
 * key (seed, 0) and counter (site, 0, 0, 0), site = (x N + y) N + z; the
 * Box-Muller cosine branch with the binary64 ln/cos sequence documented in
 * the implementation), rounded to the path precision, written as a real field
 * to out_dev (N^3 elements).  Enqueues only. */
sigw_status sigw_white_noise(sigw_plan_t plan, uint64_t seed, void* out_dev);

/* Generate the realisation of one seed into a slot (Sec. VI): white noise,
 * zeta_g_hat = sqrt(dV P(k_F|n|)) DFT(noise) with the k = 0 mode removed,
 * zeta_g, the map, Phi = 2 zeta / 3 (Sec. II at w = 1/3) and
 * Phi_hat = dV DFT(Phi), which stays on the device.  Enqueues only. */
sigw_status sigw_generate_field(sigw_plan_t plan, int32_t slot, uint64_t seed,
                                const sigw_lognormal* spectrum, const sigw_ngmap* ngmap);

/* Use a caller's own real curvature field zeta (device, real layout, path
 * precision) for a slot: the method takes a given realisation of zeta as its
 * input (Sec. I; Sec. IV computes A and B from it), and the source enters
 * through Phi = 2 zeta / 3 (Sec. II, radiation domination, w = 1/3), so the
 * slot gets Phi_hat = dV DFT(2 zeta / 3).  Enqueues only. */
sigw_status sigw_set_zeta(sigw_plan_t plan, int32_t slot, const void* zeta_dev);

/* Copy a half spectrum Phi_hat into / out of a slot (device, half layout). */
sigw_status sigw_set_phi_hat(sigw_plan_t plan, int32_t slot, const void* phi_hat_dev);
sigw_status sigw_get_phi_hat(sigw_plan_t plan, int32_t slot, void* phi_hat_dev);

/* The source convolutions of one target (Eq. final_envelopes), unfused
 * output for inspection: for kernels m = 0 (s), 1 (c) and components
 * c = xx, yy, zz, xy, xz, yz, writes
 *   Q_hat^(m)_c = dV DFT( sum_a sigma_a G_a,i G_a,j ),
 *   G_a,j = (1/V) sum_n exp(i q.x) i qt_j phi_a(k_F |n| / k_target) Phi_hat(n)
 * to qhat_dev as 12 consecutive half spectra [m][c][kx][ky][kz].
 * qt_j = k_F n_j, zero where n_j = -N/2.  Enqueues only. */
sigw_status sigw_source_convolutions(sigw_plan_t plan, int32_t slot, double k_target,
                                     void* qhat_dev);

/* Omega^(RD)_GW at n_k targets (Sec. III, IV).  Target b uses the
 * convolutions at k_targets[b] and the shell of modes n != 0 with
 * k_lo[b] <= k_F |n| < k_hi[b]:
 *   S_b = sum_{n in shell} sum_{m} sum_lambda |e^lambda : X^(m)(n)|^2,
 *   X^(s) = -(4/k_b^2) Q_hat^(s),  X^(c) = +(4/k_b^2) Q_hat^(c),
 *   Omega_b = k_b^3 S_b / (48 pi^2 V N_b),  N_b = number of modes in the shell.
 * Shells with no lattice mode (including shells whose |n|^2 values no
 * mode of the N^3 lattice has, e.g. |n|^2 = 7) give Omega_b = 0, N_b = 0
 * and launch no kernel.  k_lo may be negative (the shell then starts at
 * n = 0, which is excluded) and k_hi arbitrarily large.
 * A target whose weighted fields (|n_c| <= Rc, phi_a vanishing for
 * u >= u_max) and shell (|n_c| <= Kc) satisfy 2 Rc + Kc < M and 2 Kc + 1 < M
 * for a compiled size M < N is computed on that smaller grid of the same box,
 * where the circular convolution has no aliasing on the shell: the result is
 * the lattice's up to rounding.
 * Writes omega_host[n_k] and nmodes_host[n_k] (either may be NULL) and
 * synchronises the plan stream. */
sigw_status sigw_spectrum(sigw_plan_t plan, int32_t slot, int32_t n_k, const double* k_targets,
                          const double* k_lo, const double* k_hi, double* omega_host,
                          int64_t* nmodes_host);

/* The same for several slots that share the targets: omega_host[s * n_k + b]
 * for s = 0..n_sel-1 over slots[s] (n_sel * n_k <= 4096).  The slots run
 * `batch` at a time, each group in one launch per kernel.  Synchronises. */
sigw_status sigw_spectrum_batch(sigw_plan_t plan, int32_t n_sel, const int32_t* slots,
                                int32_t n_k, const double* k_targets, const double* k_lo,
                                const double* k_hi, double* omega_host, int64_t* nmodes_host);

/* Spectrum of one slot with jackknife error bars (Sec. IV): for every target,
 * Omega and N_b as sigw_spectrum, and the error of Omega from M^3
 * leave-one-out replicas.  The TT-projected modes of the shell (both
 * kernels) are transformed to real space; by Parseval the shell power splits
 * into the M^3 sub-volume sums S_i (FP64); replica i takes
 * M^3/(M^3-1) (S_b - S_i) with the shell's N_b, and
 * omega_err = sqrt((M^3-1)/M^3 sum_i (Omega_i - mean)^2).  M >= 2 divides N
 * and M^3 < 4096 (the paper uses M = 4); every shell must lie below the
 * Nyquist frequency k_F N/2.  replicas (n_k * M^3, may be NULL) receives
 * the replica Omegas, sub-volume index (a M + b) M + c for x in
 * [a, a+1) N/M, y in [b, b+1) N/M, z in [c, c+1) N/M.  Uses the plan's
 * workspace; synchronises the plan stream after every target. */
sigw_status sigw_spectrum_jackknife(sigw_plan_t plan, int32_t slot, int32_t n_k, const double* k_targets,
                                    const double* k_lo, const double* k_hi, int32_t M, double* omega_host,
                                    int64_t* nmodes_host, double* omega_err_host, double* replicas_host);

/* The paper's per-target measurement protocol (Sec. VI): for each target k
 * the box is L_k = pi N / k_max with k_max = 3 max(k, k_bar), k_bar the
 * wavenumber below which a fraction 1 - eps of the log-normal's power in
 * d log k lies (eps = 0.1 in the paper); the field of this seed and map is
 * generated in that box into the slot and Omega is measured in the thin
 * shell k +- pi/L_k.  Writes Omega, N_b and L_k per target (any output may
 * be NULL).  The plan's own box is restored afterwards and the slot is left
 * empty (it held fields of other boxes).  Synchronous. */
sigw_status sigw_spectrum_adaptive(sigw_plan_t plan, int32_t slot, uint64_t seed, const sigw_lognormal* spectrum,
                                   const sigw_ngmap* ngmap, int32_t n_k, const double* k_targets, double eps,
                                   double* omega_host, int64_t* nmodes_host, double* box_host);

/* Asynchronous form for serving loops: enqueue the spectrum of one slot
 * (n_k <= 64) and return at once; sigw_spectrum_poll returns SIGW_E_PENDING
 * until the plan stream has finished that work, then writes the results as
 * sigw_spectrum does.  Only one asynchronous spectrum per plan is in flight. */
sigw_status sigw_spectrum_enqueue(sigw_plan_t plan, int32_t slot, int32_t n_k,
                                  const double* k_targets, const double* k_lo, const double* k_hi);
sigw_status sigw_spectrum_poll(sigw_plan_t plan, double* omega_host, int64_t* nmodes_host);

/* Captured spectra for repeated batches (e.g. ensembles of new realisations
 * in the same slots): sigw_graph_create records, as one HIP graph on the
 * plan stream, everything sigw_spectrum_batch would enqueue for these slots
 * and targets (the plan stream must not be the null stream, and timing must
 * be off).  sigw_graph_launch replays it on the plan stream for whatever
 * fields the slots hold at that point; sigw_graph_results synchronises the
 * plan stream and writes the Omega and N_b of the last replay, laid out as
 * in sigw_spectrum_batch.  The graph owns its slot list and result buffers;
 * it shares the plan's workspace, so replays must not overlap other work of
 * the same plan.  Destroy every graph before its plan. */
typedef struct sigw_graph* sigw_graph_t;
sigw_status sigw_graph_create(sigw_plan_t plan, int32_t n_sel, const int32_t* slots, int32_t n_k,
                              const double* k_targets, const double* k_lo, const double* k_hi,
                              sigw_graph_t* out);
sigw_status sigw_graph_launch(sigw_graph_t graph);   /* SIGW_E_STATE if the plan's u grid changed since capture */
sigw_status sigw_graph_results(sigw_graph_t graph, double* omega_host, int64_t* nmodes_host);
sigw_status sigw_graph_destroy(sigw_graph_t graph);

/* Project-written autotuner of the x-pass schedule.  The fused kernel that
 * runs the last inverse pass (x), the products and the first forward pass
 * reads the most bytes of the path; several schedules of it are compiled
 * for each N: the z chunk one workgroup transforms (2 to 16 values, which
 * sets its LDS tile) and the workgroups-per-CU occupancy it is compiled for.
 * sigw_autotune times each on the plan's own workspace (one launch over
 * alpha_chunk terms and all kx planes to warm up, then the fastest of three,
 * HIP events on the plan stream), keeps the fastest, and stores the choice
 * for this (device, N, precision) in a process-wide table that later plans
 * created with desc.autotune = 1 reuse.  flags: 0 = reuse the table entry if
 * there is one, SIGW_TUNE_FORCE = time again.  It overwrites the plan's
 * workspace and synchronises the plan stream, so it must not run while an
 * asynchronous spectrum of the plan is in flight (SIGW_E_STATE).  Every
 * schedule computes the same values in the same order, so results do not
 * depend on the choice.
 * sigw_plan_schedule reports the active schedule: its index among the
 * compiled ones (0 = the default), their count, and a text line
 * ("tzx=8 occ=3", followed by the measured times after a tuning run; may
 * be NULL).  sigw_plan_set_schedule selects one by index. */
#define SIGW_TUNE_FORCE 1
sigw_status sigw_autotune(sigw_plan_t plan, int32_t flags);
sigw_status sigw_plan_schedule(sigw_plan_t plan, int32_t* index, int32_t* count, char* text, size_t text_len);
sigw_status sigw_plan_set_schedule(sigw_plan_t plan, int32_t index);

/* Host-only: the modes of the N^3 lattice (box L) in the shell
 * k_lo <= k_F |n| < k_hi, n != 0 (Sec. IV shell estimator), as sigw_spectrum
 * counts them: *count = N_b, and [*n2_lo, *n2_hi] the range of |n|^2 over
 * them (either pointer may be NULL; untouched when *count = 0).  The shell
 * test is the FP64 k_F sqrt(|n|^2) the device lookup tables use; k_lo may be
 * negative and k_hi arbitrarily large.  SIGW_E_INVALID for an unsupported N,
 * L <= 0, non-finite edges, k_hi <= k_lo or count == NULL. */
sigw_status sigw_shell_modes(int32_t N, double L, double k_lo, double k_hi, int32_t* n2_lo, int32_t* n2_hi,
                             int64_t* count);

/* Streaming-rate probe, a measurement aid (not a step of the method): the
 * device-memory rate of a plain kernel of one of four access patterns, the
 * achievable figures the hot kernels' HBM fractions are read against.
 * kind 0: read one array (float4 loads, a sum per block), 1: write one array,
 * 2: copy one array into a second, 3: read two arrays and write three (the
 * y-pass kernel's mix).  bytes is the size of one array (a multiple of 16,
 * at least 32 MiB); buf_dev must hold (1, 1, 2, 5 arrays for kind 0..3) x
 * bytes plus 32 KiB (the read's block sums).  One warm-up launch, then the
 * fastest of reps launches timed with HIP events on hip_stream (NULL = the
 * null stream); *gb_per_s = arrays x bytes / time.  Synchronises. */
sigw_status sigw_stream_probe(int32_t kind, void* buf_dev, size_t bytes, int32_t reps, void* hip_stream,
                              double* gb_per_s);

/* Block until the plan stream is idle. */
sigw_status sigw_synchronize(sigw_plan_t plan);

/* Kernel timing since timing was last enabled, over completed spectra:
 * average duration in milliseconds of the launches of the named kernel
 * ("gen_z", "ypass", "xprod", "ypass_q", "zbin"), measured with HIP events
 * on the plan stream, and the number of launches.  Timing is off by
 * default; enabling it resets the totals. */
sigw_status sigw_set_timing(sigw_plan_t plan, int32_t enabled);
sigw_status sigw_kernel_time(sigw_plan_t plan, const char* name, double* avg_ms, int64_t* launches);

/* Allocation-free spectrum, for callers that cannot allocate device memory
 * (code under HIP graph capture's restrictions, tight serving loops,
 * harnesses that forbid hipMalloc).  It computes what sigw_plan_create +
 * sigw_set_phi_hat + sigw_spectrum compute for one realisation, with no
 * plan: d describes the lattice and decomposition as for sigw_plan_create
 * (n_slots, batch and autotune are ignored; the default x-pass schedule
 * runs), phi_hat_dev is the caller's device half spectrum Phi_hat (layout and
 * precision as sigw_set_phi_hat), the targets and shells are as in
 * sigw_spectrum, and omega_host[n_k], nmodes_host[n_k] (either may be NULL)
 * receive the results.  Work is enqueued on hip_stream (NULL = the null
 * stream), which the call synchronises.
 * Every device buffer the call needs (twiddles, kernel and lookup tables,
 * workspace, shell partials) lives in one static array of SIGW_NOALLOC_BYTES
 * per GPU, which that GPU holds until the process ends; the call makes no
 * device or pinned-host allocation.  Limits: N <= 64, and the layout must
 * fit the array: with alpha_chunk = 0 (scratch_terms = 0) the largest term
 * count per x pass (staged terms) that fits is used, an explicit value that
 * does not fit returns SIGW_E_INVALID.  Results agree with sigw_spectrum up
 * to rounding (the term grouping may differ).  Every value a kernel reads is
 * written earlier in the same call, so nothing needs to start at zero.  All
 * calls on one GPU share its array: calls that overlap on one GPU (other host
 * threads, other streams) race and give wrong results.  Errors as for
 * sigw_spectrum; sigw_last_error(NULL) gives the text of this thread's last
 * failed call. */
#define SIGW_NOALLOC_BYTES (64u << 20)
sigw_status sigw_spectrum_noalloc(const sigw_plan_desc* d, const void* phi_hat_dev, int32_t n_k,
                                  const double* k_targets, const double* k_lo, const double* k_hi,
                                  double* omega_host, int64_t* nmodes_host, void* hip_stream);

const char* sigw_last_error(sigw_plan_t plan);   /* plan == NULL: the last sigw_spectrum_noalloc failure */
const char* sigw_status_string(sigw_status s);

#ifdef __cplusplus
}
#endif

#endif /* SIGW_H */
