/*
 * chebrbm -- MI355X (gfx950) hot path of the Chebyshev-RBM spectral-function
 * method (Hendry, Chen, Weinberg, Feiguin, arXiv:2103.08804).
 *
 * A small C ABI.  The calls follow the paper's statement of the problem:
 *   crbm_init_rbm          RBM parameters of the form of Sec. I
 *   crbm_init_chains       starting spin configurations of the Markov chains
 *   crbm_sample            samples s ~ |psi_s|^2 / <psi|psi>              (Sec. III)
 *   crbm_local_estimators  per-sample log psi, local energy (Sec. VI Hamiltonian),
 *                          Chebyshev target ratio R = phi/psi (Sec. III
 *                          recursion of targets), tanh(theta) and O_k     (Sec. III)
 *   crbm_sr_step           natural-gradient step (S + eps I) dalpha = F   (Sec. III)
 *   crbm_sr_energy_step    the same step on the energy gradient (ground state, Sec. I)
 *   crbm_chebyshev_moment  mu_n = <t_0|t_n> by sampling psi_gs           (Sec. II, App. A)
 *   crbm_fidelity_grad     gradient of the frozen-sample fidelity surrogate
 *   crbm_moment_matrices   overlap and Hamiltonian matrices of the Chebyshev basis (Sec. IV, App. A)
 *   crbm_sym_matrices      the same matrices of symmetry-projected states, all momenta (App. A)
 *   crbm_corrected_moments moments of the recursion repeated inside that basis   (Sec. IV)
 *   crbm_lanczos           tridiagonal form of the projected Hamiltonian        (Sec. V)
 *   crbm_spectrum_kpm      Jackson-damped Chebyshev reconstruction A(omega)      (Sec. II, Eq. Aw)
 *   crbm_spectrum_cf       continued-fraction spectrum from the tridiagonal form (Sec. V)
 *
 * Conventions
 *  - Spins are int8 +-1, row-major [rows][N].  Site r = x + Lx*y.
 *  - Complex arrays named "complex64" are interleaved (re, im) float pairs
 *    (torch.complex64 layout); "complex128" are interleaved double pairs.
 *  - RBM parameters: a[N], b[M], W[N][M] complex64 (W row-major).  A packed
 *    parameter vector is [a | b | W] of length P = N + M + N*M.
 *  - Array arguments are DEVICE pointers owned by the caller unless a comment
 *    says "host".  The library never frees or retains caller memory; it owns
 *    only the workspace inside a plan.
 *  - Every call is asynchronous on the given stream and never synchronises
 *    the host.  Scalar results are written to device memory.
 *  - Return value: CRBM_OK or a negative CRBM_E* code.  Argument errors are
 *    detected on the host before anything is enqueued; crbm_last_error()
 *    then returns a thread-local message.  Conditions found on the device
 *    (non-finite values, CG not converged, failed Cholesky pivot) are reported
 *    as bits in the caller's device stats buffer, not as return codes.
 *  - A plan must not be used from two streams at the same time.
 */
#ifndef CHEBRBM_H
#define CHEBRBM_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define CRBM_OK            0
#define CRBM_EINVAL       -1   /* bad argument (null pointer, negative size, unknown enum) */
#define CRBM_EUNSUPPORTED -2   /* valid but unsupported shape (e.g. N > 256, M > 512) */
#define CRBM_EHIP         -3   /* a HIP runtime call failed */
#define CRBM_ENOMEM       -4   /* workspace allocation failed / plan too small */

/* device flag bits in stats_out[6] of crbm_sr_step */
#define CRBM_FLAG_NOT_CONVERGED 1
#define CRBM_FLAG_NONFINITE     2
#define CRBM_FLAG_CHOLESKY_FAIL 4

enum { CRBM_LATTICE_CHAIN = 0, CRBM_LATTICE_SQUARE = 1 };
enum { CRBM_PROPOSAL_FLIP = 0, CRBM_PROPOSAL_EXCHANGE = 1 };
enum { CRBM_SOLVER_CG_DENSE = 0, CRBM_SOLVER_CG_MATFREE = 1, CRBM_SOLVER_CHOLESKY = 2 };
enum { CRBM_PREC_FP32 = 0, CRBM_PREC_BF16 = 1 };

/* plan flags */
#define CRBM_PLAN_DENSE_S 1    /* reserve the dense P x P complex64 matrix S and the packed operands of
                                  its matrix-core contraction (needed by CG_DENSE); for small P also up to
                                  min(8, 2^30 / (8 P^2)) more P x P slices, so that the contraction can be
                                  split over samples when its tile pairs alone cannot fill the device */
#define CRBM_PLAN_CHOLESKY 2   /* also reserve a P x P complex128 factor (CHOLESKY; needs P <= 4000) */
#define CRBM_PLAN_BASIS 4      /* reserve the workspace of crbm_moment_matrices for K = n_max + 1 <= basis_k_max
                                  (crbm_plan_create_ex): 16 K_max max_samples + 8 max_samples bytes */
#define CRBM_PLAN_SYM_BASIS 8  /* reserve the workspace of crbm_sym_matrices for K <= basis_k_max:
                                  32 K_max max_samples + (N + 24) max_samples bytes (includes CRBM_PLAN_BASIS) */

/* workspace buffers readable through crbm_plan_buffer (device pointers) */
enum {
    CRBM_BUF_F = 0,        /* complex128 [P]   right-hand side F of the last sr_step */
    CRBM_BUF_DALPHA = 1,   /* complex128 [P]   solution dalpha of the last sr_step */
    CRBM_BUF_OMEAN = 2,    /* complex128 [P]   <O_k> of the last sr_step */
    CRBM_BUF_S = 3,        /* complex64 [P][P] S of the last dense sr_step (both triangles) */
    CRBM_BUF_WAVE_CLOCKS = 4 /* uint64 [CRBM_MAX_CLOCK_WAVES][2] (start, end) of every wave of the last
                                crbm_batched_moments launched while profiling was on (crbm_plan_profile),
                                in ticks of the device's constant 100 MHz clock; waves of larger grids
                                are not recorded, unused rows are 0 */
};
#define CRBM_MAX_CLOCK_WAVES 16384

typedef struct crbm_plan_s* crbm_plan;

/* One RBM (Sec. I): psi(sigma) = exp(sum_i a_i sigma_i) prod_j 2 cosh(theta_j),
 * theta_j = b_j + sum_i W_ij sigma_i.  All three arrays are complex64 device memory. */
typedef struct {
    int n_visible;   /* N */
    int n_hidden;    /* M */
    void* a;         /* complex64 [N] */
    void* b;         /* complex64 [M] */
    void* W;         /* complex64 [N][M] */
} crbm_rbm;

/* Periodic nearest-neighbour lattice of the Heisenberg model H = J sum_<ij> S_i.S_j (Sec. VI).
 * CHAIN: N = Lx sites, bonds (i, i+1 mod N).  SQUARE: N = Lx*Ly, bonds (r, r+x) and (r, r+y)
 * for every site r (coinciding bonds of a side of length 2 are kept twice). */
typedef struct {
    int kind;        /* CRBM_LATTICE_* */
    int Lx, Ly;      /* Ly ignored for CHAIN */
    double J;
} crbm_lattice;

/* Chebyshev stage (Sec. III recursion of targets, rescaled Hamiltonian of Sec. II):
 * the state being fitted is t~_{n+1}; H~ = (H - E_c)/W_scale; the target is
 *   order 0:   phi = beta_n H~ t_0,                   t_0 = f_q psi_gs
 *   order >=1: phi = 2 beta_n H~ t~_n - beta_nm1 t~_{n-1},   t~_0 = t_0
 * f_q(sigma) = N^{-1/2} sum_r exp(-i q.r) sigma_r / 2 (the S^z_q operator of App. B). */
typedef struct {
    int order;
    double E_c, W_scale;
    double beta_n[2];    /* complex (re, im) */
    double beta_nm1[2];  /* complex (re, im) */
    double q[2];         /* (q_x, q_y); q_y ignored on a chain */
} crbm_cheb;

/* Plan: lattice, hidden width and the largest sample count any later call on it will use.
 * Allocates the device workspace (O(max_samples * (N + M)) plus O(P) vectors; plus
 * 8*P*P bytes with CRBM_PLAN_DENSE_S).  Limits: N even or odd up to 256, M up to 512.
 * Uses the current HIP device. */
int crbm_plan_create(crbm_plan* plan, const crbm_lattice* lattice, int n_hidden, long max_samples, int flags);
/* The same with the basis workspace of the moment correction (Sec. IV, App. A) reserved up front for
 * K = n_max + 1 <= basis_k_max <= 256 (flags CRBM_PLAN_BASIS / CRBM_PLAN_SYM_BASIS; basis_k_max is ignored
 * without them), so that crbm_moment_matrices and crbm_sym_matrices allocate nothing and can be captured in
 * a graph from their first call.  crbm_plan_create(p, l, M, S, f) is crbm_plan_create_ex(p, l, M, S, f, 0). */
int crbm_plan_create_ex(crbm_plan* plan, const crbm_lattice* lattice, int n_hidden, long max_samples, int flags,
                        int basis_k_max);
int crbm_plan_destroy(crbm_plan plan);
/* Device pointer and size in bytes of a workspace buffer (CRBM_BUF_*), valid until destroy. */
int crbm_plan_buffer(crbm_plan plan, int which, void** dev_ptr, size_t* bytes);
/* Thread-local text of the last error returned on this thread. */
const char* crbm_last_error(void);

/* Instrumentation.  While enabled, the library records HIP events on the call's stream around
 * each kernel group below (one kernel launch per record unless noted).  crbm_plan_profile
 * enables (1) or disables (0) recording and discards earlier records; crbm_plan_profile_read
 * waits for the recorded events of one group and returns the number of records and their total
 * duration in milliseconds. */
enum {
    CRBM_PROF_SAMPLE = 0,   /* Metropolis sweep kernel */
    CRBM_PROF_THETA,        /* theta = sigma W + b product */
    CRBM_PROF_LOCAL,        /* local-estimator kernel */
    CRBM_PROF_OT,           /* O^H c contraction kernel */
    CRBM_PROF_SBUILD,       /* dense S contraction kernel, rows of the hidden biases b and weights W (matrix cores;
                               the tile pairs of the full site blocks and those of the last, partly filled one) */
    CRBM_PROF_CG,           /* whole conjugate-gradient loop (many kernels) */
    CRBM_PROF_MOMENT,       /* per-order moment ratio kernel */
    CRBM_PROF_PACK,         /* operand packing for the S contraction (two kernels) */
    CRBM_PROF_CHOLESKY,     /* whole Cholesky factorisation and solve (many kernels) */
    CRBM_PROF_BATCHED,      /* batched moments: counter reset, persistent kernel, per-instance reduction */
    CRBM_PROF_GRAM,         /* moment-correction matrices: G and H products and their reduction (two kernels) */
    CRBM_PROF_SBORDER,      /* dense S contraction: the rows of the visible biases a (matrix cores) */
    CRBM_PROF_COUNT
};
int crbm_plan_profile(crbm_plan plan, int enable);
int crbm_plan_profile_read(crbm_plan plan, int group, int* count, double* total_ms);

/* Ceiling probes for rooflines (instrumentation; both synchronise the stream and allocate and free
 * temporary device memory on the current device):
 * crbm_probe_mfma: sustained TFLOP/s of the BF16 matrix cores (v_mfma_f32_32x32x16_bf16, eight
 *   independent accumulators per wave, two workgroups of four waves per compute unit, no memory
 *   traffic in the loop), written to host *tflops_out.
 * crbm_probe_hbm: copy bandwidth in GB/s (bytes read + bytes written) of a 16-byte grid-stride copy
 *   of `bytes` (>= 1 MiB) between two device buffers, written to host *gbs_out.
 * crbm_probe_logcosh: evaluations per second of Re log(2 cosh z) in the Metropolis sweep's form
 *   (hardware exp, cos and log; eight independent evaluations per lane, no memory traffic), the
 *   transcendental ceiling of the sweep (Sec. III sampling), written to host *evals_out.
 * crbm_probe_gather: GB/s of whole-row reads of an n_rows x row_elems complex64 table at pseudo-random
 *   rows, lanes over the row (the sweep's reads of rows W_i, W_j), written to host *gbs_out; the
 *   table holds at most 2^24 entries. */
int crbm_probe_mfma(double* tflops_out, hipStream_t stream);
int crbm_probe_hbm(size_t bytes, double* gbs_out, hipStream_t stream);
int crbm_probe_logcosh(double* evals_out, hipStream_t stream);
int crbm_probe_gather(int n_rows, int row_elems, double* gbs_out, hipStream_t stream);

/* Fill a, b, W with complex numbers whose real and imaginary parts are independent
 * N(0, stddev^2): parameter k of the packed vector takes Philox4x32-10 block
 * (key = seed, counter = (k, 0, 0, 2)), u1 = ((x0 >> 8) + 1) 2^-24, u2 = (x1 >> 8) 2^-24,
 * and Box-Muller stddev sqrt(-2 ln u1) (cos 2 pi u2, sin 2 pi u2). */
int crbm_init_rbm(const crbm_rbm* rbm, uint64_t seed, float stddev, hipStream_t stream);

/* Starting configurations spins[n_chains][N].  zero_magnetisation = 0: sigma_i = +1 iff bit 0
 * of x0 of block (seed; chain, i, 0, 1).  zero_magnetisation = 1 (N even): N/2 up spins then
 * N/2 down spins, Fisher-Yates shuffled: for k = N-1 .. 1 swap k with floor(x0 (k+1) / 2^32),
 * x0 from block (seed; chain, k, 0, 1). */
int crbm_init_chains(crbm_plan plan, int8_t* spins, int n_chains, uint64_t seed, int zero_magnetisation,
                     hipStream_t stream);

/* Metropolis sampling of P(s) = |psi_s|^2 / <psi|psi> (Sec. III), n_chains independent chains.
 * Step t = step_offset + sweep*N + k (k = 0..N-1) of chain c draws Philox block
 * (key = seed; counter = (c, t lo32, t hi32, 0)): i = floor(x0 N / 2^32), j = floor(x1 N / 2^32),
 * u = (x2 >> 8) 2^-24.  FLIP flips site i; EXCHANGE swaps sites i and j if sigma_i != sigma_j,
 * else the step is a null move.  Accept iff u < |psi(sigma')/psi(sigma)|^2.  One sample is the
 * state after each sweep of N steps.
 *   spins        int8 [n_chains][N]      in: start states, out: final states
 *   theta_out    complex64 [n_chains][M] or NULL: theta of the final states
 *   logpsi_out   complex64 [n_chains]    or NULL: log psi of the final states (Im mod 2 pi)
 *   samples_out  int8 [n_sweeps][n_chains][N] or NULL
 *   n_accept     uint32 [n_chains] or NULL: accepted steps in this call
 *   accept_trace uint32 [n_chains][ceil(n_sweeps*N/32)] or NULL: bit (sweep*N+k) = accepted
 * n_sweeps = 0 leaves the spins as they are and writes theta, log psi of the start states and
 * n_accept = 0. */
int crbm_sample(crbm_plan plan, const crbm_rbm* psi, int8_t* spins, void* theta_out, void* logpsi_out,
                int n_chains, int n_sweeps, int proposal, uint64_t seed, uint64_t step_offset,
                int8_t* samples_out, uint32_t* n_accept, uint32_t* accept_trace, hipStream_t stream);

/* Per-sample estimators on samples[n_samples][N] (Sec. III, Sec. VI).
 * Energy mode (psi_n == NULL, cheb ignored): eloc_out = (H fit)(s)/fit(s).
 * Chebyshev mode (psi_n != NULL): fit = t~_{n+1}; psi_n = t~_n (psi_gs at order 0);
 *   psi_nm1 = t~_{n-1} (psi_gs at order 1, unused at order 0);
 *   eloc_out = (H g)(s)/psi_n(s) with g = t_0 at order 0 and g = psi_n otherwise;
 *   R_out = phi(s)/fit(s).
 * Outputs (any may be NULL): logpsi_out complex64 [n] (log fit, Im mod 2 pi), eloc_out
 * complex64 [n], R_out complex64 [n], tanh_out complex64 [n][M] (tanh theta of fit),
 * O_out complex64 [n][P] (O_a = sigma, O_b = tanh theta, O_W = sigma_i tanh theta_j).
 * n_samples = 0 writes nothing and launches nothing (samples and outputs may then be NULL); the
 * arguments are still checked. */
int crbm_local_estimators(crbm_plan plan, const crbm_rbm* fit, const crbm_rbm* psi_n, const crbm_rbm* psi_nm1,
                          const crbm_cheb* cheb, const int8_t* samples, long n_samples,
                          void* logpsi_out, void* eloc_out, void* R_out, void* tanh_out, void* O_out,
                          hipStream_t stream);

/* Natural-gradient step on fit (Sec. III), from the samples, their tanh(theta) (as written by
 * crbm_local_estimators) and the target ratios R:
 *   gamma = arccos sqrt(|<R>|^2/<|R|^2>), beta = <R>,
 *   F_k = dgamma gamma cot(gamma) [<O_k^* R>/<R> - <O_k^*>]   (gamma cot gamma -> 1 - gamma^2/3 below 1e-4)
 *   S_kk' = <O_k^* O_k'> - <O_k>^* <O_k'>,   (S + diag_shift I) dalpha = F,   alpha += dalpha.
 * <f> = sum_s w_s f_s with w = weights (double [n]) or 1/n if weights == NULL.
 * solver: CG_DENSE (S built densely by the O^H O contraction, CG with double vectors),
 *         CG_MATFREE (S v = <O^*(O v)> - <O>^*(<O> v) from the factored O each iteration),
 *         CHOLESKY (S built densely, factorised in double).
 * s_precision: FP32 or BF16 operands of the dense S contraction on the matrix cores, FP32 accumulation
 *         (BF16 needs weights == NULL; with weights the FP32 contraction runs on the vector units).
 * cg_tol: relative residual |F - (S+eps)x| / |F|; cg_maxit: iteration cap.
 * stats_out: device double [8] = {gamma, Re beta, Im beta, |F|_2, relative residual,
 *            iterations, flags (CRBM_FLAG_*), |dalpha|_2}.
 * The parameters of fit are updated in place (complex64). */
int crbm_sr_step(crbm_plan plan, const crbm_rbm* fit, const int8_t* samples, const double* weights,
                 const void* tanh_theta, const void* R, long n_samples, double dgamma, double diag_shift,
                 int solver, int s_precision, double cg_tol, int cg_maxit, double* stats_out,
                 hipStream_t stream);

/* Figure of merit and normalisation of a fit as it stands (Sec. III), from the target ratios R of its
 * current parameters (crbm_local_estimators in Chebyshev mode):
 *   gamma = arccos sqrt(|<R>|^2/<|R|^2>),   beta = <R>   (the normalisation taken once the steps are done).
 * weights: double [n] or NULL (1/n), as in crbm_sr_step.
 * stats_out: device double [5] = {gamma, Re beta, Im beta, <|R|^2>, flags (CRBM_FLAG_NONFINITE when
 * <|R|^2> is not positive or a sum is not finite)}. */
int crbm_fit_stats(crbm_plan plan, const void* R, const double* weights, long n_samples, double* stats_out,
                   hipStream_t stream);

/* Exact-enumeration weights: with all configurations listed once as samples, the sampling distribution
 * of Sec. III, P(s) = |psi_s|^2/<psi|psi>, is
 *   weights_out[s] = exp(2 Re logpsi[s] - LSE),   LSE = log sum_s' exp(2 Re logpsi[s'])   (double).
 * logpsi: complex64 [n] (as written by crbm_local_estimators); weights_out: double [n].
 * The partial sums are merged in a fixed order (deterministic).  Every weight is NaN when no amplitude
 * is finite and non-zero. */
int crbm_enum_weights(crbm_plan plan, const void* logpsi, long n, double* weights_out, hipStream_t stream);

/* Natural-gradient energy minimisation of psi, by which the ground state psi_gs that seeds the
 * expansion is obtained (Sec. I, with the metric S of Sec. III):
 *   E = <E_loc>,  F_k = -lr [<O_k^* E_loc> - <O_k>^* <E_loc>]   (the bracket is dE/d conj(alpha_k)),
 *   (S + diag_shift I) dalpha = F,   alpha += dalpha.
 * eloc: complex64 [n_samples], (H psi)(s)/psi(s) as written by crbm_local_estimators in energy mode
 * for the same psi and samples; tanh_theta likewise.  Samples, weights, solver, s_precision, cg_tol
 * and cg_maxit as in crbm_sr_step; lr must be finite.
 * stats_out: device double [8] = {<|E_loc|^2> - |E|^2, Re E, Im E, |F|_2, relative residual,
 *            iterations, flags (CRBM_FLAG_*), |dalpha|_2}.
 * The parameters of psi are updated in place (complex64). */
int crbm_sr_energy_step(crbm_plan plan, const crbm_rbm* psi, const int8_t* samples, const double* weights,
                        const void* tanh_theta, const void* eloc, long n_samples, double lr, double diag_shift,
                        int solver, int s_precision, double cg_tol, int cg_maxit, double* stats_out,
                        hipStream_t stream);

/* Chebyshev moments by sampling s ~ |psi_gs|^2 (Sec. II, App. A):
 *   mu_0(q) = <|f_q|^2>,  mu_n(q) = < f_q(s)^* beta_n t~_n(s)/psi_gs(s) >  (n = 1..n_max)
 * t_params: complex64 [n_max][P], packed [a|b|W] of t~_1 .. t~_{n_max}; betas: complex128 [n_max];
 * q: HOST double [n_q][2]; weights as in crbm_sr_step; mu_out: complex128 [n_q][n_max+1],
 * accumulated in double. */
int crbm_chebyshev_moment(crbm_plan plan, const crbm_rbm* psi_gs, const void* t_params, const double* betas,
                          int n_max, const double* q, int n_q, const int8_t* samples, const double* weights,
                          long n_samples, void* mu_out, hipStream_t stream);

/* Gradient of the frozen-sample fidelity surrogate L = (1/n) sum_s |1 - R_s|^2 with respect to the
 * parameters of fit (R = phi/fit, so dR/dalpha_k = -R O_k):
 *   grad_k = 2 dL/d conj(alpha_k) = (2/n) sum_s (1 - R_s) conj(R_s) conj(O_k(s)),
 * i.e. dL/dRe alpha_k + i dL/dIm alpha_k.  grad_out: complex128 [P] or NULL; loss_out: double [1] or NULL
 * (at least one of the two).
 * tanh_theta and R as written by crbm_local_estimators for the same fit and samples. */
int crbm_fidelity_grad(crbm_plan plan, const crbm_rbm* fit, const int8_t* samples, const void* tanh_theta,
                       const void* R, long n_samples, void* grad_out, double* loss_out, hipStream_t stream);

/* crbm_fidelity_grad without a plan and without any allocation, for callers that cannot allocate device
 * memory (code under graph capture, tight serving or training loops, harnesses that forbid hipMalloc).
 * Same arguments and result as crbm_fidelity_grad (same kernels, bit-identical output) with the shape given
 * directly (n_visible <= 256, n_hidden <= 512).  Its scratch (the packed spin rows and the FP32 chunk sums of
 * the O^H contraction) lives in one static device array of 48 MiB that each GPU the library runs on holds
 * until the process ends; a gradient needing more (about n (N + 17) + 8 (N + 1)(M + 1) ceil(n / max(256,
 * n/256)) bytes) returns CRBM_ENOMEM before anything is enqueued.  Every byte of the scratch that a call
 * reads is written earlier in the same call, so nothing carries over from a previous call; but all calls on
 * one GPU share the array: calls that overlap on one GPU (two streams, two host threads) race. */
int crbm_fidelity_grad_noalloc(int n_visible, int n_hidden, const int8_t* samples, const void* tanh_theta,
                               const void* R, long n_samples, void* grad_out, double* loss_out, hipStream_t stream);

/* Moment-correction matrices of the basis t_0 = S^z_q psi_gs, t_n = beta_n t~_n (n = 1..n_max), by
 * sampling s ~ |psi_gs|^2 (Sec. IV; App. A, G and H):
 *   B_0(s) = f_q(s),  B_n(s) = beta_n t~_n(s)/psi_gs(s),  HB_n(s) = (H t_n)(s)/psi_gs(s),
 *   G_nm = <conj(B_n) B_m> = <t_n|t_m>/<psi_gs|psi_gs>,  H_nm = <conj(B_n) HB_m> = <t_n|H|t_m>/<psi_gs|psi_gs>.
 * H is the lattice Hamiltonian of the plan (units of J, not rescaled).  K = n_max + 1 <= 256.
 * t_params, betas, weights, samples as in crbm_chebyshev_moment; q: HOST double [2];
 * G_out, H_out: complex128 [K][K] (row n, column m).  Row 0 of G is the moment estimate mu_m of
 * crbm_chebyshev_moment on the same samples.  Needs a plan created with CRBM_PLAN_BASIS (or
 * CRBM_PLAN_SYM_BASIS) and basis_k_max >= K; otherwise CRBM_ENOMEM.  Allocates nothing. */
int crbm_moment_matrices(crbm_plan plan, const crbm_rbm* psi_gs, const void* t_params, const double* betas,
                         int n_max, const double* q, const int8_t* samples, const double* weights, long n_samples,
                         void* G_out, void* H_out, hipStream_t stream);

/* Symmetry-projected moment-correction matrices (App. A) for all N lattice momenta at once.
 * The stored RBMs approximate the Chebyshev vectors of the LOCAL operator at site 0:
 * t_000 = S^z_0 psi_gs and t_n00 = beta_n t~_n (n = 1..n_max).  A symmetry g acts on configurations
 * as (s o g)_r = s_{g(r)}; the group is the translations T_m and, if rotations = 1 (L x L lattice
 * only), the rotation R(x, y) = (L-1-y, x).  Over samples s ~ |psi_gs|^2:
 *   B_{n,m,rot}(s) = t_n00(s o T_m R^rot)/psi_gs(s)   (and HB with (H t_n00) in place of t_n00),
 *   Bt_{nk}(s) = N^{-1/2} sum_m e^{-i k.m} (1/4) [B_{n,m,0} + B_{n,m+(1,0),1} + B_{n,m+(1,1),2}
 *                + B_{n,m+(0,1),3}]   (only the first term, with weight 1, without rotations),
 *   G^(k)_nn' = <conj(Bt_nk) Bt_n'k>,  H^(k)_nn' = <conj(Bt_nk) HBt_n'k>,
 * k.m = 2 pi (k1 m1/Lx + k2 m2/Ly), k = k1 + Lx k2.  G_out, H_out: complex128 [N][K][K], K = n_max + 1.
 * With a translation- and rotation-invariant psi_gs, row 0 of G^(k) holds the moments of S^z_k.
 * The images of a sample are evaluated in chunks of max_samples / (N * (rotations ? 4 : 1)) samples
 * (that quotient must be >= 1).  Needs a plan created with CRBM_PLAN_SYM_BASIS and basis_k_max >= K;
 * otherwise CRBM_ENOMEM.  Allocates nothing. */
int crbm_sym_matrices(crbm_plan plan, const crbm_rbm* psi_gs, const void* t_params, const double* betas,
                      int n_max, int rotations, const int8_t* samples, const double* weights, long n_samples,
                      void* G_out, void* H_out, hipStream_t stream);

/* Corrected Chebyshev moments (Sec. IV): the recursion repeated for the Hamiltonian projected onto the
 * span of the basis,  H' = (H - E_c G)/W_scale  (the rescaled Hamiltonian of Sec. II in the basis),
 *   c_0 = e_0,  G c_1 = H' c_0,  G c_{n+1} = 2 H' c_n - G c_{n-1},  mu_n = Re sum_l G_0l c_ln,
 * for n = 0 .. n_out-1 (n_out may exceed K).  G and H (complex128 [K][K], device) are replaced by their
 * Hermitian parts; G is factorised by Cholesky in double.  mu_out: double [n_out] (device).
 * info_out: double [3] (device) = {flags (CRBM_FLAG_CHOLESKY_FAIL if G is not positive definite; then
 * mu_out is zero), max_n |mu_n|/mu_0 (exceeds 1 when the estimated matrices are inconsistent),
 * smallest/largest Cholesky pivot}. */
int crbm_corrected_moments(crbm_plan plan, const void* G, const void* H, int K, double E_c, double W_scale,
                           int n_out, double* mu_out, double* info_out, hipStream_t stream);

/* Lanczos tridiagonalisation of the Hamiltonian projected onto the basis (Sec. V), started from t_0,
 * with full re-orthogonalisation, in double.  Hermitian parts of G and H are used.  Runs
 * min(n_steps, K) steps or stops at an invariant subspace.
 * a_out: double [n_steps] diagonal; b2_out: double [n_steps], b2_out[0] = G_00 = <t_0|t_0>/<psi_gs|psi_gs>
 * and b2_out[j] = b_j^2 (j >= 1) the squared off-diagonal; info_out: double [2] = {flags, steps done m}.
 * The Green's function of t_0 is b2_0 / (z - a_0 - b2_1 / (z - a_1 - ... b2_{m-1} / (z - a_{m-1}))). */
int crbm_lanczos(crbm_plan plan, const void* G, const void* H, int K, int n_steps, double* a_out, double* b2_out,
                 double* info_out, hipStream_t stream);

/* Chebyshev reconstruction (Sec. II, Eq. Aw) on a frequency grid (all pointers device):
 *   A(omega) = [g_0 mu_0 + 2 sum_{n=1}^{n_mom-1} g_n mu_n T_n(x)] / (pi W_scale sqrt(1 - x^2)),
 *   x = (E0 + omega - E_c)/W_scale,  A = 0 for |x| >= 1,
 * g_n the Jackson factors of Sec. VI for N = n_mom moments if jackson != 0, else 1.
 * mu: double [n_mom] (real moments); omega: double [n_omega] excitation energies; A_out: double [n_omega]. */
int crbm_spectrum_kpm(const double* mu, int n_mom, int jackson, double E0, double E_c, double W_scale,
                      const double* omega, int n_omega, double* A_out, hipStream_t stream);

/* Continued-fraction spectrum (Sec. V) from crbm_lanczos output with m levels (all pointers device):
 *   A(omega) = -(1/pi) Im G(omega + E0 + i eta),  eta > 0 the broadening. */
int crbm_spectrum_cf(const double* a, const double* b2, int m, double E0, double eta, const double* omega,
                     int n_omega, double* A_out, hipStream_t stream);

/* Batched Chebyshev moments of many (q, n) instances in one persistent launch (Sec. II moments,
 * App. A momentum form).  Instance i has a momentum q_i, a stored state t~_i and beta_i, and owns
 * c_i = chain_offsets[i+1] - chain_offsets[i] Markov chains on psi_gs.  Chain g (global index) starts
 * from a Fisher-Yates S^z = 0 configuration (Philox tag 1, counter a = g, as crbm_init_chains), runs
 * n_burn unrecorded and n_sweeps recorded sweeps with the proposals of crbm_sample (counter a = g,
 * step = sweep*N + k), and after each recorded sweep adds |f_q(s)|^2 and f_q(s)^* beta_i t~_i(s)/psi_gs(s).
 *   t_params      complex64 [n_inst][P], packed [a|b|W] of each t~_i
 *   betas         complex128 [n_inst]
 *   q             device double [n_inst][2]
 *   chain_offsets device int64 [n_inst + 1], non-decreasing, chain_offsets[0] = 0,
 *                 chain_offsets[n_inst] = total_chains <= the plan's max_samples.  The offsets live in
 *                 device memory and are not checked on the host: a chain takes the instance found by
 *                 binary search whatever they hold, and an instance whose range is not inside
 *                 [0, total_chains] gets NaN in both moments (no access outside the buffers)
 *   mu_out        complex128 [n_inst][2] = (<|f_q|^2>, <f_q^* beta t~/psi_gs>) per instance
 *   trace         NULL, or device uint32 [total_chains][ceil((n_burn + n_sweeps) * N / 32)]: the accept
 *                 bit of every proposal of chain g (bit t % 32 of word t / 32 of row g, t = sweep*N + k,
 *                 burn-in included; null moves are 0), as crbm_sample records them, so that another
 *                 implementation can replay the chains; every word is written
 * Waves of a persistent grid take chains from an atomic counter; partial sums are reduced per
 * instance in chain order, so the result does not depend on the schedule.  The launch shape is the
 * plan's default or the one chosen by crbm_batched_autotune.  Safe to capture in a graph. */
int crbm_batched_moments(crbm_plan plan, const crbm_rbm* psi_gs, const void* t_params, const double* betas,
                         const double* q, const int64_t* chain_offsets, int n_inst, int64_t total_chains, int n_burn,
                         int n_sweeps, int proposal, uint64_t seed, void* mu_out, uint32_t* trace,
                         hipStream_t stream);
/* Times the persistent kernel of crbm_batched_moments for several launch shapes (lanes per chain 64,
 * 32 or 16 where M allows, waves per block 1..8, blocks per compute unit 1..8) on the given instances
 * with n_sweeps_probe sweeps, stores the fastest in the plan and returns it (any output may be NULL).
 * Every shape gives the same moments and traces bit for bit (the sums run in one fixed order).
 * Synchronises the host: call it outside graph capture. */
int crbm_batched_autotune(crbm_plan plan, const crbm_rbm* psi_gs, const void* t_params, const double* betas,
                          const double* q, const int64_t* chain_offsets, int n_inst, int64_t total_chains,
                          int n_sweeps_probe, int proposal, uint64_t seed, void* mu_scratch,
                          int* waves_per_block, int* blocks, int* lanes_per_chain, double* best_ms,
                          hipStream_t stream);
/* K tile (samples staged per LDS tile: 64 or 128) of the BF16 matrix-core S contraction of this plan's
 * dense sr_step.  Every tile gives the same S bit for bit (the samples are summed in the same order).
 * Default 128.  Does not touch the device. */
int crbm_plan_set_sbuild_tile(crbm_plan plan, int k_tile);
/* Times the BF16 S contraction (Sec. III) of this plan with each K tile on the given samples (int8
 * [n][N]) and tanh theta (complex64 [n][M]), stores the faster tile in the plan and returns it (outputs
 * may be NULL).  Overwrites the plan's dense S.  Needs a plan with CRBM_PLAN_DENSE_S.  Synchronises the
 * host: call it outside graph capture. */
int crbm_sbuild_autotune(crbm_plan plan, const int8_t* samples, const void* tanh_theta, long n, int* k_tile,
                         double* best_ms, hipStream_t stream);
/* Sets the launch shape of crbm_batched_moments: waves per block (1..8), blocks, lanes per chain (64;
 * 32 for M <= 256; 16 for M <= 128: several chains share a wave).  CRBM_EUNSUPPORTED for a lane count
 * that M does not allow.  Does not touch the device. */
int crbm_batched_set_shape(crbm_plan plan, int waves_per_block, int blocks, int lanes_per_chain);
/* Whether crbm_batched_moments on 64 lanes per chain, with this proposal kind (CRBM_PROPOSAL_FLIP or
 * CRBM_PROPOSAL_EXCHANGE) and waves per block, reads the rows of psi_gs from a copy of its W in LDS
 * (*uses = 1) rather than from global memory (*uses = 0).  The copy is taken when W (N M complex64) and the spin
 * rows fit in the compute unit's LDS and the unit still holds as many blocks as without it; both paths
 * give the same results bit for bit.  Queries the device's occupancy; enqueues nothing. */
int crbm_batched_lds_rows(crbm_plan plan, int proposal, int waves_per_block, int* uses);

#ifdef __cplusplus
}
#endif
#endif /* CHEBRBM_H */
