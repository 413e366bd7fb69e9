// Internal launch interface between the C-ABI layer and the kernel
// translation units.  Every launcher enqueues on `stream` and returns the
// hipError_t of the launch.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "profile.hpp"

namespace crbm {

struct RbmView {            // device pointers, complex64 interleaved
    const float2* a;
    const float2* b;
    const float2* W;
};

// theta = sigma W + b (complex64 [n][M]) on the matrix cores; planes: lc_plane_elems(N, M) scratch for
// the split W; skip (device, may be null) != 0 makes both launches return at once
hipError_t launch_theta(const int8_t* sig, long n, int N, int M, const float2* b, const float2* W, float2* theta,
                        uint16_t* planes, hipStream_t stream, const double* skip = nullptr);
// O v of the matrix-free S product, u[s] = sum_k T_sk (sigma_s V_W + v_b)_k + sigma_s . v_a, without
// writing the n x M product; partial: n * ceil(M / 64) double2 scratch
hipError_t launch_theta_ov(const int8_t* sig, long n, int N, int M, const float2* vb, const float2* vW,
                           const double2* va, const float2* T, uint16_t* planes, double2* partial, double2* u,
                           hipStream_t stream, const double* skip);

// elements of the three BF16 planes of W used by the theta product and the fused log-cosh sums: 3 x (tiles of 64 units x 128
// real columns) x (sites rounded up to 32)
inline long lc_plane_elems(long N, long M) { return 3L * ((M + 63) / 64) * 128L * ((N + 31) / 32 * 32); }

// bonds of the largest lattice (square, N <= 256 sites, 2 N bonds); the local-estimator kernel keeps
// a per-wave list of the anti-aligned ones in LDS
constexpr int kMaxBonds = 512;
// row length of the packed sigma~ of the O^H c contraction: sites 0..N-1, then 1 (b), then zeros
inline int sig16_row(int N) { return ((N + 1 + 15) / 16) * 16; }

struct Geometry {
    int N, M, P;
    int n_bonds;
    const int2* bonds;      // device [n_bonds]
    int kind, Lx;           // for site positions (f_q phases)
    double J;
    float4* bond_tab;       // device [n_bonds][M] workspace: (exp 2D, exp -2D), D = W_i - W_j of one RBM
    uint8_t* node_flag;     // device [max_samples] workspace: 1 where the local-energy RBM is next to a node
};

// ---------------------------------------------------------------- init
hipError_t launch_init_rbm(float2* a, float2* b, float2* W, int N, int M, uint64_t seed, float stddev,
                           hipStream_t stream);
hipError_t launch_init_chains(int8_t* spins, int N, int n_chains, uint64_t seed, int zero_mag, hipStream_t stream);

// ---------------------------------------------------------------- sampling
struct SampleArgs {
    RbmView psi;
    int N, M;
    int8_t* spins;
    float2* theta_out;
    float2* logpsi_out;
    int n_chains, n_sweeps, proposal;
    uint64_t seed, step_offset;
    int8_t* samples_out;
    uint32_t* n_accept;
    uint32_t* trace;
    int trace_words;
};
hipError_t launch_sample(const SampleArgs& args, hipStream_t stream);

// ---------------------------------------------------------------- local estimators
struct LocalArgs {
    Geometry g;
    RbmView fit, psn, psm;  // psn.a == nullptr -> energy mode; psm unused at order 0
    int cheb_mode;
    int local_op;           // Chebyshev mode: t_0 = S^z_0 psi (local operator at site 0) instead of S^z_q psi
    int order;
    double E_c, W_scale;
    double2 beta_n, beta_nm1;
    float2 lbeta_n, lbeta_nm1;   // log beta_n, log beta_nm1 (principal branch; beta = 0 gives Re = -inf)
    double q0, q1;
    const int8_t* samples;
    long n_samples;
    float2* logpsi_out;
    float2* eloc_out;
    float2* R_out;
    float2* tanh_out;
    float2* O_out;
};
hipError_t launch_local(const LocalArgs& args, hipStream_t stream);

// ---------------------------------------------------------------- moments
struct MomentArgs {
    Geometry g;
    RbmView gs;
    const float2* t_params;   // [n_max][P]
    const double2* betas;     // [n_max]
    int n_max;
    const double* q;          // device [n_q][2]
    int n_q;
    const int8_t* samples;
    const double* weights;
    long n_samples;
    double2* partial;         // workspace [n_blocks][n_q][n_max + 1]
    int n_blocks;
    double2* mu_out;          // [n_q][n_max + 1]
};
hipError_t launch_moments(const MomentArgs& args, hipStream_t stream);

// ---------------------------------------------------------------- natural-gradient step
struct SrWork {
    double* scal;             // [32] device scalars (see kernels_sr.hip)
    double2* Om;              // [P]  <O>
    double2* Om16;            // [P]  <O> of the operands of the matrix-core S contraction (shifted, rounded)
    double2* ORm;             // [P]  <O^* (R - <R>)> (R = E_loc in energy mode)
    double2* F;               // [P]
    double2* x;               // [P]  solution
    double2* r;               // [P]
    double2* p;               // [P]
    double2* Ap;              // [P]
    double2* u;               // [n]  per-sample scratch for the matrix-free product
    double2* red;             // reduction scratch [red_len]
    long red_len;
    float2* S;                // [P][P] dense (may be null)
    double2* S64;             // [P][P] dense double (Cholesky, may be null)
    float2* G;                // [n][2 ceil(M / 64)] scratch of the matrix-free product (its O v partials)
    int8_t* sig16;            // [n][sig16_row(N)] sigma~ rows for the O^H c contraction
    float2* vstage;           // [P] float copy of a CG direction
    void* pack;               // packed operand planes of the matrix-core S contraction
    size_t pack_bytes;
    const int2* sb_order;     // dispatch order of its tile pairs (full tiles, then the ragged pairs)
    long sb_order_len;
    float2* spart;            // [nsplit_max][P][P] partial sums of a contraction split over samples (or null)
    float2* bx;               // [N][P] raw a-row sums of the matrix-core S contraction
    float2* bx_part;          // [nsplit_max][N][P] their split partial sums (with spart)
    double2* hv_part;         // [nT][nT][kHemvTile] tile shares of the dense Hermitian product (with S)
    uint16_t* wplanes;        // split-W scratch of the theta product (the matrix-free product's G)
    int nsplit_max;
    int nsb_max;              // slices of bx_part: sample splits of the border kernel (1: none)
    int sb_kt;                // K tile (samples) of the BF16 S contraction: 64 or 128
    int n_cu;
    Profiler* prof;
};

// instrumentation group ids (mirrors CRBM_PROF_* of the public header)
enum { PROF_SAMPLE = 0, PROF_THETA, PROF_LOCAL, PROF_OT, PROF_SBUILD, PROF_CG, PROF_MOMENT, PROF_PACK, PROF_CHOLESKY,
       PROF_BATCHED, PROF_GRAM, PROF_SBORDER, PROF_COUNT };

struct SrArgs {
    int N, M, P;
    float2* a; float2* b; float2* W;   // fit parameters (updated in place)
    const int8_t* samples;
    const double* weights;             // may be null
    const float2* T;                   // tanh theta [n][M]
    const float2* R;                   // [n]
    long n;
    double dgamma, eps;
    int solver, prec;
    double cg_tol;
    int cg_maxit;
    double* stats;                     // device [8]
    int mode;                          // 0: Chebyshev fit (R = target ratio); 1: energy (R = E_loc, dgamma = -lr)
};
// edge of the square tiles of the dense Hermitian product and its number of tile rows for P parameters
constexpr int kHemvTile = 256;
inline int hemv_tiles(long P) { return (int)((P + kHemvTile - 1) / kHemvTile); }

// the dense FP64 solve is meant for P of a few thousand (its factor is P^2 complex128 values)
constexpr long kCholMaxP = 4000;

hipError_t launch_sr_step(const SrArgs& args, const SrWork& w, hipStream_t stream);

// ---------------------------------------------------------------- batched moments
struct BatchedArgs {
    int N, M, P, kind, Lx;
    RbmView gs;
    const float2* t_params;      // [n_inst][P]
    const double2* betas;        // [n_inst]
    const double* q;             // [n_inst][2]
    const int64_t* offsets;      // [n_inst + 1]
    int n_inst;
    int64_t total;
    int n_burn, n_sweeps, proposal;
    uint64_t seed;
    unsigned long long* counter;
    double2* partial;            // [total][2]
    uint32_t* trace;             // [total][trace_words] accept bits, or null
    int trace_words;
    unsigned long long* clocks;  // [CRBM_MAX_CLOCK_WAVES][2] (start, end) per wave, or null
};
// the matrix-core S contraction (kernels_mfma.hip); kt_bf16: K tile of the BF16 variant, 64 or 128
hipError_t launch_sbuild_mfma(int N, int M, long P, const int8_t* sig, const float2* T, long n,
                              const double2* shift, const double2* Om, float2* S, int prec, int kt_bf16, void* pack,
                              size_t pack_bytes, const int2* order, long n_order, float2* split_buf, int nsplit,
                              float2* bx, float2* bx_part, int nsb, Profiler* prof,
                              hipStream_t stream);
int sbuild_splits(int N, int M, long n, int n_cu, int max_splits);
int sbuild_border_splits(int N, int M, long n, int n_cu, int max_splits);

// lanes per chain: 64 (any M), 32 (M <= 256) or 16 (M <= 128); the results are the same bit for bit
bool batched_lanes_ok(int lanes, int M);
bool batched_lds_rows(int N, int M, int proposal, int waves_per_block);
hipError_t launch_batched(const BatchedArgs& A, int blocks, int waves_per_block, int lanes, double2* mu,
                          hipStream_t stream);
// p[0, n) = 0 with a fill kernel (no memset node when captured)
hipError_t launch_clear_u64(unsigned long long* p, long n, hipStream_t stream);

struct GradArgs {
    int N, M, P;
    const int8_t* samples;
    const float2* T;
    const float2* R;
    long n;
    double2* grad;                     // [P]
    double* loss;                      // [1] or null
};
hipError_t launch_fidelity_grad(const GradArgs& args, const SrWork& w, hipStream_t stream);
// the same gradient with its scratch (fidelity_grad_scratch_bytes(N, M, n) bytes) supplied by the caller
size_t fidelity_grad_scratch_bytes(int N, int M, long n);
hipError_t launch_fidelity_grad_scratch(const GradArgs& args, void* scratch, int n_cu, hipStream_t stream);

// gamma, beta = <R>, <|R|^2> and a flag word of the current fit (out: device double [5]); red: 512 double2
hipError_t launch_fit_stats(const float2* R, const double* w, long n, double2* red, double* out, hipStream_t stream);
// p(s) = exp(2 Re log psi_s - LSE) over n listed configurations; part: kLseParts double2 scratch
constexpr int kLseParts = 256;
hipError_t launch_enum_weights(const float2* logpsi, long n, double2* part, double* w, hipStream_t stream);

}  // namespace crbm
