/*
 * pfsh.h -- C ABI of the MI355X (gfx950) hot path of PFASST-SH: the IMEX SDC
 * sweep of the rotating shallow-water equations in a spherical-harmonic basis
 * (Hamon, Schreiber & Minion, "Parallel-in-Time Multi-Level Integration of the
 * Shallow-Water Equations on the Rotating Sphere").
 *
 * Conventions shared by every call
 * --------------------------------
 * Truncation T (triangular): zonal wavenumber m = 0..T, total wavenumber
 * n = m..T; K = (T+1)(T+2)/2 coefficients per field, stored m-major
 * (slot of (m,n) = m(T+1) - m(m-1)/2 + (n-m)).  Only m >= 0 is stored: the
 * fields are real, so the m<0 coefficients are conjugates and Im of every m=0
 * coefficient is 0 (Sec. 3).  Legendre functions are normalized to
 * int_{-1}^{1} (P_n^m)^2 dmu = 1 with P_m^m > 0.
 *
 * Spectral arrays are complex128, real and imaginary parts interleaved.
 *   state       [batch][3][K]            variables (Phi, zeta, delta)  (Sec. 2)
 *   space-time  [batch][n_nodes][3][K]   SDC nodes 0..M               (Sec. 5.1.1)
 * Grid arrays are float64 [field][nlat][nlon]: Gaussian latitudes from north to
 * south (mu = sin(latitude) descending), longitudes lambda_k = 2 pi k/nlon.
 *
 * Ownership: every array argument is a DEVICE pointer owned by the caller
 * (allocated e.g. through PyTorch) unless it is marked "host".  A level owns its
 * tables and its workspace, sized by max_batch at creation; no call allocates
 * device memory after creation (pfsh_pfasst_create allocates its own buffers).
 *
 * Asynchrony and errors: every compute call only enqueues kernels on `stream`
 * (a hipStream_t passed as void*; NULL = the null stream) and returns at once.
 * Arguments are validated on the host before anything is enqueued; a rejected
 * call enqueues nothing.  Launch failures are reported as PFSH_EHIP.  Nothing
 * throws across the ABI.  One level object may be used by one stream at a time
 * (its workspace is shared by all of its calls).
 */
#ifndef PFSH_H
#define PFSH_H

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PFSH_OK = 0,
  PFSH_EINVAL = -1,       /* null pointer, bad scalar argument */
  PFSH_ESHAPE = -2,       /* sizes inconsistent (batch > max_batch, grid too coarse, ...) */
  PFSH_ENOMEM = -3,       /* device allocation failed at creation */
  PFSH_EHIP = -4,         /* a HIP runtime call or kernel launch failed */
  PFSH_EUNSUPPORTED = -5, /* valid but not implemented (e.g. nlon not 2^a or 3*2^a)     */
  PFSH_ENONFINITE = -6    /* a NaN/Inf was found (pfsh_check_finite) */
} pfsh_status;

/* Arithmetic of the transform stages (Legendre contractions, ring FFTs, grid
 * products).  The spectral pre/post steps, the implicit solve, the SDC
 * accumulation, the residual and the transfers are FP64 in every mode. */
typedef enum {
  PFSH_FP64 = 0,   /* FP64 tables and data, FP64 MFMA                        */
  PFSH_FP32 = 1,   /* FP32 tables and data, FP32 MFMA, FP32 accumulate       */
  PFSH_BF16X3 = 2  /* x = hi + lo with hi = bf16(x), lo = bf16(x - hi) for
                      table and data; products hi*hi + hi*lo + lo*hi on BF16
                      MFMA with FP32 accumulate; FFT and products in FP32     */
} pfsh_precision;

/* Flag OR-ed into pfsh_level_desc.precision (FP64 and FP32 only): the level
 * stores no Legendre tables.  The Legendre contractions generate the
 * normalized P_n^m(mu_j) they need inside the kernel, in FP64, by the
 * three-term recurrence in n (Sec. 3; the on-the-fly evaluation of the
 * transform the paper builds on) taken two degrees at a time so that each
 * parity runs on its own:
 *   P_{n+2} = ((mu^2 - e_{n+1}^2 - e_n^2) P_n - e_n e_{n-1} P_{n-2}) / (e_{n+1} e_{n+2}),
 *   e_n = sqrt((n^2 - m^2) / (4 n^2 - 1)),
 * restarted every 32 degrees of one parity from two stored values (about 1/8
 * of the FP32 table's size), and round the values to the transform type for
 * the MFMA operands.  Results agree with the tabulated mode to the rounding
 * of the recurrence (about 1e-14 relative in FP64).  The batch-1/2 fused node
 * kernel needs the tables, so such a level runs small batches on the separate
 * kernels.  Invalid (PFSH_EINVAL) with PFSH_BF16X3. */
#define PFSH_LEGENDRE_RECURRENCE 0x100

/* One space-time level of the hierarchy (Sec. 5.3). */
typedef struct {
  int T;          /* triangular truncation (largest wavenumber), 1 <= T <= 767         */
  int nlat;       /* Gaussian latitudes: even, >= T+2                                  */
  int nlon;       /* longitudes: >= 2T+2, of the form 2^a or 3*2^a, 16 <= nlon <= 1536 */
  int n_nodes;    /* Gauss-Lobatto SDC nodes M+1, 2..9 (the paper uses 2, 3 and 5)     */
  int max_batch;  /* largest batch (time slices x members) any call will use, >= 1     */
  double radius;  /* sphere radius a [m]                                               */
  double omega;   /* rotation rate Omega [1/s]; Coriolis f = 2 Omega mu               */
  double phibar;  /* mean geopotential Phibar [m^2/s^2]                                */
  double nu;      /* diffusion coefficient nu [m^2/s]                                  */
  int precision;  /* pfsh_precision of the transform stages, | PFSH_LEGENDRE_RECURRENCE */
} pfsh_level_desc;

typedef struct pfsh_level pfsh_level;

/* Human-readable name of a status code (static string, never NULL). */
const char* pfsh_status_string(pfsh_status s);

/* Host-only validation of a descriptor (no HIP call).  PFSH_OK if
 * pfsh_level_create would accept it; PFSH_EINVAL / PFSH_ESHAPE /
 * PFSH_EUNSUPPORTED otherwise. */
pfsh_status pfsh_level_desc_check(const pfsh_level_desc* desc);

/* Create a level on `device`: Gaussian grid, normalized Legendre tables up to
 * degree T+1 (built in 80-bit extended precision on the host, then rounded and
 * packed in the MFMA operand order of the chosen precision; with
 * PFSH_LEGENDRE_RECURRENCE the recurrence's restart values and coefficients
 * instead), FFT twiddles, the
 * SDC matrices Q, qE, qI of Sec. 5.1.1 and a workspace for max_batch.
 * *out receives the handle (NULL on failure).  Synchronous. */
pfsh_status pfsh_level_create(const pfsh_level_desc* desc, int device, pfsh_level** out);

/* Free a level (synchronizes its device first).  NULL is a no-op. */
void pfsh_level_destroy(pfsh_level* level);

/* Host copies of the level's sizes and SDC tables (any pointer may be NULL):
 * K, n_nodes; nodes[n_nodes] on [0,1]; q, qe, qi as row-major
 * [n_nodes][n_nodes] matrices (Sec. 5.1.1: integration matrix Q, forward-Euler
 * qE, qI = U^T of the LU factorization of Q^T restricted to nodes 1..M);
 * mu[nlat] and w[nlat]: Gaussian latitudes (north to south) and weights. */
pfsh_status pfsh_level_query(const pfsh_level* level, int* K, int* n_nodes, double* nodes,
                             double* q, double* qe, double* qi, double* mu, double* w);

/* Device memory of a level in bytes (either pointer may be NULL): *tables =
 * the Legendre tables, or in recurrence mode the restart pairs and
 * coefficients that replace them; *workspace = the transform and sweep
 * workspace sized for max_batch.  Host-only. */
pfsh_status pfsh_level_bytes(const pfsh_level* level, unsigned long long* tables,
                             unsigned long long* workspace);

/* Scalar SH synthesis (Sec. 3, eq. spectral_to_physical_space):
 * spec [nfields][K] complex128 -> grid [nfields][nlat][nlon] float64,
 * xi(lambda_k, mu_j) = sum_{m,n} xi_n^m P_n^m(mu_j) e^{i m lambda_k} (m<0 terms by
 * conjugation).  1 <= nfields <= 4*max_batch. */
pfsh_status pfsh_sh_synthesis(pfsh_level* level, const void* spec, void* grid, int nfields,
                              void* stream);

/* Scalar SH analysis (Sec. 3: Fourier transform in longitude, then Gauss-
 * Legendre quadrature in latitude): grid [nfields][nlat][nlon] float64 ->
 * spec [nfields][K] complex128, xi_n^m = sum_j w_j P_n^m(mu_j) X_m(mu_j) with
 * X_m(mu_j) = (1/nlon) sum_k xi(lambda_k, mu_j) e^{-i m lambda_k}; Im of m = 0
 * is set to 0.  1 <= nfields <= 5*max_batch. */
pfsh_status pfsh_sh_analysis(pfsh_level* level, const void* grid, void* spec, int nfields,
                             void* stream);

/* Right-hand sides at `batch` states (Sec. 2 and 4): f_expl = F_E = N(state),
 * the nonlinear terms of eq. nonlinear_operators evaluated with the transform
 * method, and f_impl = F_I = L(state) of eq.
 * linear_wave_motion_induced_by_gravitational_forces.  All [batch][3][K].
 * Either output may be NULL to skip it. */
pfsh_status pfsh_rhs(pfsh_level* level, const void* state, void* f_expl, void* f_impl, int batch,
                     void* stream);

/* Implicit solve of Sec. 5.4: x = (I - beta L)^{-1} b per mode (a 2x2 system
 * for (Phi, delta) and a scalar one for zeta).  b, x: [batch][3][K]; x may
 * equal b (in place).  beta >= 0. */
pfsh_status pfsh_implicit_solve(pfsh_level* level, double beta, const void* b, void* x, int batch,
                                void* stream);

/* One IMEX SDC sweep (Sec. 5.1.1, eq. update_equation_sdcq_discrete_form; with
 * tau != NULL the FAS form eq. modified_update_equation_sdcq_discrete_form).
 * theta, f_expl, f_impl, tau: [batch][n_nodes][3][K].  On entry node 0 holds
 * the initial condition and its F_E, F_I (already evaluated there); nodes
 * 1..M hold the previous iterate.  On return nodes 1..M hold the new iterate
 * and its F_E, F_I; node 0 is not touched.  dt > 0. */
pfsh_status pfsh_sdc_sweep(pfsh_level* level, double dt, void* theta, void* f_expl, void* f_impl,
                           const void* tau, int batch, void* stream);

/* Form of the implicit step of every sweep on the level (Sec. 5.1.1, last
 * paragraph).  PFSH_IMPLICIT_COMBINED (the default): one solve
 * (I - beta L) Theta = b per node and mode, as eq.
 * update_equation_sdcq_discrete_form is written.  PFSH_IMPLICIT_SPLIT: two
 * substeps as in the paper's implementation (multi-implicit SDC): with
 * L = L1 + L2, L1 the physical linear terms (-Phibar delta, 0, -lap Phi) and L2
 * = nu lap, Theta* = (I - beta L1)^{-1} (b + beta L2 Theta_old) and then
 * Theta = (I - beta L2)^{-1} (Theta* - beta L2 Theta_old), Theta_old the
 * previous iterate at the node, beta = dt qI_{m+1,m+1}; the same collocation
 * fixed point.  Host-only; affects sweeps enqueued (or graphs captured) after
 * the call.  PFSH_EINVAL for another mode. */
#define PFSH_IMPLICIT_COMBINED 0
#define PFSH_IMPLICIT_SPLIT 1
pfsh_status pfsh_level_set_implicit(pfsh_level* level, int mode);

/* Collocation residual (Sec. 5.1.1, eq. collocation_problem; FAS form of
 * Sec. 5.1.2 when tau != NULL): r^m = theta^0 + dt (Q F)_m + tau^m - theta^m.
 * out [batch][3] float64 (device) receives max over nodes and modes of |r|
 * per slice and variable; a NaN/Inf anywhere gives NaN in that entry. */
pfsh_status pfsh_residual(pfsh_level* level, double dt, const void* theta, const void* f_expl,
                          const void* f_impl, const void* tau, double* out, int batch, void* stream);

/* Allocation-free variant of pfsh_residual, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation): the same kernels and the same result, with the
 * per-block partial maxima in a static device array of
 * PFSH_RESIDUAL_SCRATCH_DOUBLES doubles (4 MiB) that the library holds on
 * every GPU it runs on until the process ends, instead of the level's
 * workspace.  Nothing is allocated or freed by the call.  The partials need
 * batch * 3 * ceil(K / 256) doubles; a larger request returns PFSH_ESHAPE
 * before anything is enqueued (batch may exceed the level's max_batch, the
 * call does not use the level's workspace; batch <= 65535).  All calls on one
 * GPU share the array: calls that overlap in time on one GPU (two streams, two
 * threads) race and must be ordered by the caller.  Arguments and output as
 * pfsh_residual. */
#define PFSH_RESIDUAL_SCRATCH_DOUBLES (1 << 19)
pfsh_status pfsh_residual_noalloc(pfsh_level* level, double dt, const void* theta,
                                  const void* f_expl, const void* f_impl, const void* tau,
                                  double* out, int batch, void* stream);

/* Synchronous check of a [count] float64 device array: PFSH_ENONFINITE if any
 * entry is NaN/Inf, PFSH_OK otherwise (waits for `stream`). */
pfsh_status pfsh_check_finite(const double* values, int count, void* stream);

/* Copy node 0 of theta, f_expl, f_impl to every node ("spread" initial iterate;
 * any array may be NULL).  [batch][n_nodes][3][K]. */
pfsh_status pfsh_spread(pfsh_level* level, void* theta, void* f_expl, void* f_impl, int batch,
                        void* stream);

/* Restriction R = (R^s)(R^t) of Sec. 5.3 (eq. time_restriction then
 * eq. space_restriction): in_f [batch][Mf+1][3][Kf] -> out_c [batch][Mc+1][3][Kc];
 * temporal Lagrange interpolation from fine to coarse nodes (pointwise
 * injection for nested Lobatto sets), then truncation to m, n <= Tc. */
pfsh_status pfsh_restrict(const pfsh_level* fine, const pfsh_level* coarse, const void* in_f,
                          void* out_c, int batch, void* stream);

/* Interpolation P = (P^t)(P^s) of Sec. 5.3 applied to a coarse increment and
 * added: inout_f += P (new_c - old_c) (old_c may be NULL for P new_c); zero-
 * padding in space, Lagrange interpolation from coarse to fine nodes.
 * new_c, old_c [batch][Mc+1][3][Kc]; inout_f [batch][Mf+1][3][Kf]. */
pfsh_status pfsh_interpolate_add(const pfsh_level* coarse, const pfsh_level* fine, const void* new_c,
                                 const void* old_c, void* inout_f, int batch, void* stream);

/* FAS correction of Sec. 5.1.2 (eq. tau_term_level_l+1 with tau_f = 0):
 * tau_c = dt [ R (Q_f (x) I) F_f - (Q_c (x) I) F_c ], where F_c must be the coarse
 * F at R theta_f.  fe_f, fi_f [batch][Mf+1][3][Kf]; fe_c, fi_c, tau_c
 * [batch][Mc+1][3][Kc]. */
pfsh_status pfsh_fas_tau(const pfsh_level* fine, const pfsh_level* coarse, double dt,
                         const void* fe_f, const void* fi_f, const void* fe_c, const void* fi_c,
                         void* tau_c, int batch, void* stream);

/* Kernel timing (diagnostic).  While enabled on a level, every launch of the
 * listed kernels made through that level carries a pair of HIP events that
 * take the kernel's own start and end timestamps (the launch gap before it is
 * not counted).  pfsh_profile_read synchronizes on the recorded events and
 * returns the number of timed launches and the sum of their durations in
 * milliseconds since the last enable.  Enabling clears earlier records.
 * Not to be enabled while a stream is being captured into a graph. */
typedef enum {
  PFSH_K_LEG_SYNTH = 0,   /* Legendre synthesis contraction (MFMA)        */
  PFSH_K_RING = 1,        /* ring FFTs + grid products                     */
  PFSH_K_LEG_ANAL = 2,    /* Legendre analysis contraction (MFMA)          */
  PFSH_K_ASSEMBLE = 3,    /* spectral assembly of F_E (RHS calls, last
                             node of a sweep)                              */
  PFSH_K_PREP = 4,        /* transform input preparation (RHS calls)       */
  PFSH_K_SWEEP_NODE = 5,  /* sweep node: F_E assembly of the previous node,
                             old-iterate terms (node 1), update, implicit
                             solve, F_I, transform input of the new state  */
  PFSH_K_COUNT = 6
} pfsh_kernel_id;
pfsh_status pfsh_profile_enable(pfsh_level* level, int on);
pfsh_status pfsh_profile_read(pfsh_level* level, int kernel, int* launches, double* total_ms);
/* the same restricted to launches over `batch` states (batch <= 0: all) */
pfsh_status pfsh_profile_read_batch(pfsh_level* level, int kernel, int batch, int* launches,
                                    double* total_ms);

/* ---------------------------------------------------------------------------
 * Transform-kernel variants and the autotuner.  A level launches one variant
 * of each transform stage per size bucket (the batch of an RHS evaluation,
 * rounded up to a power of two, after conversion to 16-column MFMA blocks for
 * the Legendre stages); variant 0 is the built-in default.
 *   stage 0, Legendre synthesis: prefetch depth of the K loop and wave tile
 *            (FP64 / FP32: 4, 2, 8 with 32 x 32 per wave; 4, 2 with 64 x 64 per
 *            wave; 4 with the LDS exchange in two row halves; BF16x3: 2, 4);
 *   stage 1, Legendre analysis: (prefetch depth, tile shape), shape 0 = 64
 *            degrees x 64 columns per workgroup, 1 = 64 x 32 with one degree
 *            block per wave, tall = 64 x 64 with 64 x 32 per wave (FP64 /
 *            FP32, depth in 16-byte groups of the table, 4 or 2 k-blocks
 *            each: (2,0) (1,0) (4,0) (2,1) (4,1) (1,tall) (2,tall); BF16x3,
 *            depth in k-blocks: (2,0) (4,0) (2,1) (4,1));
 *   stage 2, ring FFTs + products of the RHS: largest radix 16, 8, 4 with
 *            256 threads per workgroup, radix 16 with 512 threads;
 *   stage 3, sweep path for batches of 1-2 slices on FP64 / FP32 levels:
 *            0 = one fused kernel per node and order (Legendre analysis of the
 *            previous node's products, F_E assembly, node update, Legendre
 *            synthesis) plus the ring stage, 1 = the separate kernels.  Same
 *            bits either way; not timed by the tuner.
 * The Legendre variants give bitwise identical results (same order of every
 * sum); the ring variants differ in FFT round-off only.
 * pfsh_level_autotune times every variant of the three stages at `batch`
 * (three interleaved rounds of one warm-up and `reps` launches each, HIP
 * events on `stream`, best round per variant) on the level's internal
 * workspace, and keeps for that batch's buckets the fastest variant if it
 * beats the default by at least 3%, else the default.
 * It synchronizes the stream, overwrites the level's workspace (which holds
 * nothing between calls), and returns PFSH_EUNSUPPORTED while the stream is
 * being captured; graphs captured earlier keep the variants they recorded.
 * us_out (host, nullable, 3 * PFSH_MAX_VARIANTS floats) receives the best
 * microseconds per launch at [stage * PFSH_MAX_VARIANTS + variant], stages
 * 0-2.  One level must not be tuned and used on two streams at once.
 * ------------------------------------------------------------------------- */
#define PFSH_MAX_VARIANTS 8
/* number of variants of a stage (0..3) on this level, or a negative status */
int pfsh_variant_count(const pfsh_level* level, int stage);
pfsh_status pfsh_level_set_variant(pfsh_level* level, int stage, int batch, int variant);
pfsh_status pfsh_level_get_variant(const pfsh_level* level, int stage, int batch, int* variant);
pfsh_status pfsh_level_autotune(pfsh_level* level, int batch, int reps, void* stream,
                                float* us_out);
/* The same with flags: PFSH_TUNE_COLD times each launch alone after rewriting a
 * 512 MiB buffer (allocated and freed inside the call; PFSH_ENOMEM if it cannot
 * be), so that tables and operands come from HBM as they do between the other
 * kernels of a sweep; without it the launches run back to back with hot caches.
 * Other bits: PFSH_EINVAL. */
#define PFSH_TUNE_COLD 1
pfsh_status pfsh_level_autotune_ex(pfsh_level* level, int batch, int reps, int flags, void* stream,
                                   float* us_out);

/* ---------------------------------------------------------------------------
 * Two-level PFASST on one device (Sec. 5.2).  The n_ts time steps of a block
 * ("processors" P_0..P_{n_ts-1}) and `members` independent ensemble members
 * are one batch: slice index s = step * members + member, so a step's members
 * are contiguous.  The send/receive of Algorithm 1 become device copies along
 * the batch axis; the coarse step C stays a serial chain over steps.
 * Fine arrays theta_f, fe_f, fi_f: [n_ts*members][Mf+1][3][Kf], owned by the
 * caller.  The context owns the coarse arrays, saved copies, tau and the
 * last-node snapshots (allocated at creation).
 * ------------------------------------------------------------------------- */
typedef struct pfsh_pfasst pfsh_pfasst;

/* fine->max_batch and coarse->max_batch must be >= n_ts*members. */
pfsh_status pfsh_pfasst_create(pfsh_level* fine, pfsh_level* coarse, int n_ts, int members,
                               pfsh_pfasst** out);
void pfsh_pfasst_destroy(pfsh_pfasst* ctx);

/* Prediction (Sec. 5.2.1) from theta0 [members][3][Kf]: broadcast, restrict,
 * n_ts wavefront stages of coarse sweeps (stage j sweeps steps j..n_ts-1, step
 * n >= 1 taking the stage-(j-1) last-node value of step n-1 as its initial
 * condition), then fine = spread(theta0) + P(coarse - R spread(theta0)) and
 * fine F at all nodes.  Writes theta_f, fe_f, fi_f. */
pfsh_status pfsh_pfasst_predict(pfsh_pfasst* ctx, double dt, const void* theta0, void* theta_f,
                                void* fe_f, void* fi_f, void* stream);

/* One PFASST iteration (Sec. 5.2.2, Algorithm 1): A) batched fine sweep; if
 * `last` != 0 stop here; B) restrict, coarse F at all nodes, saved copies, tau;
 * C) serial chain over steps: new coarse initial condition from step n-1,
 * coarse F at node 0, coarse FAS sweep; D) interpolate the coarse increments of
 * theta, F_E and F_I to all fine nodes, new fine initial condition = fine
 * last-node value of step n-1 from A plus P(coarse initial condition - R of that
 * value), fine F at node 0. */
pfsh_status pfsh_pfasst_iterate(pfsh_pfasst* ctx, double dt, void* theta_f, void* fe_f, void* fi_f,
                                int last, void* stream);

/* n_iter PFASST iterations (the last stopping after its fine sweep) in
 * wavefront order: super-step t advances every time step n whose iteration
 * k = t - n lies in [0, n_iter), batched over that contiguous range of steps.
 * Each step needs only what its left neighbour produced one super-step earlier
 * (the coarse last-node value of step C, the fine last-node value of step A),
 * so the serial coarse chains of consecutive iterations overlap: n_ts + n_iter
 * - 1 super-steps instead of n_iter serial chains of n_ts coarse sweeps.  The
 * arithmetic is that of n_iter pfsh_pfasst_iterate calls (bitwise for FP64).
 * If fine_alt is not NULL (same geometry as the fine level), iterations
 * k >= k_switch sweep on fine_alt, and the step-D re-evaluation of F at node
 * 0 that precedes them does too.  Replayed from a captured graph when graphs
 * are on. */
pfsh_status pfsh_pfasst_run(pfsh_pfasst* ctx, double dt, void* theta_f, void* fe_f, void* fi_f,
                            int n_iter, pfsh_level* fine_alt, int k_switch, void* stream);

/* PFASST iterations with a convergence check, the variant the paper leaves to
 * future work (Sec. 5.2.2): after the fine sweep (step A) of every iteration
 * the fine collocation residual of every slice is taken (pfsh_residual: max
 * over nodes and modes, per variable) and copied to the host; when it is at
 * most tol[v] (host, 3 absolute bounds for Phi, zeta, delta) for every slice
 * and variable, or when max_iter iterations have run, the iteration stops
 * there, after its fine sweep, as the last iteration of pfsh_pfasst_iterate
 * does; otherwise steps B-D follow.  Synchronizes the stream once per
 * iteration; direct launches (no graph replay).  iterations (host, nullable)
 * receives the number of iterations performed, residuals (host, nullable,
 * [max_iter][n_ts*members][3]) the residuals after each fine sweep.
 * PFSH_ENONFINITE when a residual is NaN/Inf (the iteration stops there). */
pfsh_status pfsh_pfasst_run_tol(pfsh_pfasst* ctx, double dt, void* theta_f, void* fe_f, void* fi_f,
                                int max_iter, const double* tol, int* iterations, double* residuals,
                                void* stream);

/* Serial comparators of Sec. 5.5 on the same kernels.
 *
 * pfsh_sdc_run: SDC(M+1, nsweeps) over nsteps time steps of dt for `batch`
 * independent states.  theta, f_expl, f_impl [batch][n_nodes][3][K]: on entry
 * node 0 of theta holds the initial states (the other entries are work
 * space); each step evaluates F at node 0, spreads state and F to every node
 * (the spread initial iterate), runs nsweeps sweeps and moves the last node to
 * node 0.  On return node 0 (and the last node) hold the states after nsteps
 * steps.
 *
 * pfsh_mlsdc_run: MLSDC(Mf+1, Mc+1, n_iter, alpha) over nsteps steps with the
 * levels of a PFASST context created with n_ts = 1 (members = the batch; else
 * PFSH_ESHAPE).  Each step starts as above on the fine level and runs n_iter
 * iterations of one fine sweep, the restriction, coarse F at all coarse nodes
 * and tau, one coarse FAS sweep from the restricted initial condition, and the
 * interpolated increments of Theta, F_E, F_I at all fine nodes (Algorithm 1 on
 * one time step); fine arrays and return as pfsh_sdc_run. */
pfsh_status pfsh_sdc_run(pfsh_level* level, double dt, void* theta, void* f_expl, void* f_impl,
                         int nsteps, int nsweeps, int batch, void* stream);
pfsh_status pfsh_mlsdc_run(pfsh_pfasst* ctx, double dt, void* theta_f, void* fe_f, void* fi_f,
                           int nsteps, int n_iter, void* stream);

/* Swap the context's fine and coarse levels for levels of the same geometry
 * (T, nlat, nlon, n_nodes, device; max_batch large enough), e.g. levels of
 * another transform precision: later calls use the new levels, the state
 * arrays are kept.  Used to finish a block with FP64 fine sweeps after
 * iterations with mixed-precision transforms. */
pfsh_status pfsh_pfasst_set_levels(pfsh_pfasst* ctx, pfsh_level* fine, pfsh_level* coarse);

/* When on, pfsh_pfasst_iterate captures the kernel sequence of an iteration
 * on its stream into a HIP graph the first time it sees a given (arrays, dt,
 * last, levels, stream) and replays it afterwards.  Needs a non-null stream
 * that is not already being captured; otherwise the kernels are launched
 * directly.  Turning it off synchronizes the device and frees the graphs. */
pfsh_status pfsh_pfasst_set_graphs(pfsh_pfasst* ctx, int on);

#ifdef __cplusplus
}
#endif
#endif /* PFSH_H */
