/*
 * FP64 CPU oracle for the Chebyshev-RBM hot path (Hendry, Chen, Weinberg,
 * Feiguin, "Chebyshev expansion of spectral functions using restricted
 * Boltzmann machines", arXiv:2103.08804).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * reference that the GPU library is checked against.  It shares no code,
 * header, table or constant generator with the HIP library; only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark may load
 * it.  The product path never calls it.
 *
 * Every quantity is computed from its definition in double precision, with no
 * incremental caching: a ratio psi(s')/psi(s) is always the exponential of two
 * log-amplitudes evaluated from scratch.
 *
 * Conventions (the paper leaves these open; the readings are listed in the
 * design notes):
 *   - visible units sigma_i in {+1,-1}, S^z_i = sigma_i / 2;
 *   - site r = x + Lx*y; enumeration index s <-> sigma_i = +1 iff bit i set;
 *   - parameter vector order [a_0..a_{N-1}, b_0..b_{M-1}, W_00, W_01, ...]
 *     (W row-major, index N + M + i*M + j);
 *   - complex numbers are interleaved (re, im) doubles.
 */
#define _GNU_SOURCE
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* ------------------------------------------------------------------------- */
/* Philox4x32-10, from Salmon, Moraes, Dror and Shaw, "Parallel random        */
/* numbers: as easy as 1, 2, 3" (SC'11): ten rounds of the 4x32 S-box with    */
/* the published multipliers and Weyl key increments.                         */
/* ------------------------------------------------------------------------- */
#define PHILOX_MULT_A 0xD2511F53u
#define PHILOX_MULT_B 0xCD9E8D57u
#define PHILOX_WEYL_A 0x9E3779B9u
#define PHILOX_WEYL_B 0xBB67AE85u

void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
    uint32_t x0 = ctr_in[0], x1 = ctr_in[1], x2 = ctr_in[2], x3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += PHILOX_WEYL_A; k1 += PHILOX_WEYL_B; }
        uint64_t pa = (uint64_t)PHILOX_MULT_A * (uint64_t)x0;
        uint64_t pb = (uint64_t)PHILOX_MULT_B * (uint64_t)x2;
        uint32_t hi_a = (uint32_t)(pa >> 32), lo_a = (uint32_t)pa;
        uint32_t hi_b = (uint32_t)(pb >> 32), lo_b = (uint32_t)pb;
        uint32_t y0 = hi_b ^ x1 ^ k0;
        uint32_t y1 = lo_b;
        uint32_t y2 = hi_a ^ x3 ^ k1;
        uint32_t y3 = lo_a;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Stream layout: key = (seed lo32, seed hi32); counter = (a, b lo32, b hi32, tag). */
static void philox_draw(uint64_t seed, uint32_t a, uint64_t b, uint32_t tag, uint32_t out[4]) {
    uint32_t ctr[4] = {a, (uint32_t)b, (uint32_t)(b >> 32), tag};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    orc_philox4x32_10(ctr, key, out);
}

/* floor(x * n / 2^32): a site index in [0, n). */
static int draw_index(uint32_t x, int n) { return (int)(((uint64_t)x * (uint64_t)n) >> 32); }
/* (x >> 8) * 2^-24: a uniform in [0, 1), exact in binary32 and binary64. */
static double draw_unit(uint32_t x) { return (double)(x >> 8) * (1.0 / 16777216.0); }

/* ------------------------------------------------------------------------- */
/* Parameter initialisation: Re and Im of every complex parameter are         */
/* independent N(0, stddev^2).  One Philox draw per parameter (tag 2,         */
/* counter a = parameter index); Box-Muller on u1 = ((x0>>8)+1)/2^24 in       */
/* (0,1] and u2 = (x1>>8)/2^24.                                               */
/* ------------------------------------------------------------------------- */
void orc_init_rbm(int N, int M, uint64_t seed, double stddev, cplx* a, cplx* b, cplx* W) {
    long P = (long)N + M + (long)N * M;
    for (long k = 0; k < P; ++k) {
        uint32_t r[4];
        philox_draw(seed, (uint32_t)k, 0, 2u, r);
        double u1 = ((double)(r[0] >> 8) + 1.0) * (1.0 / 16777216.0);
        double u2 = (double)(r[1] >> 8) * (1.0 / 16777216.0);
        double rad = stddev * sqrt(-2.0 * log(u1));
        double ang = 2.0 * M_PI * u2;
        cplx v = rad * cos(ang) + I * (rad * sin(ang));
        if (k < N) a[k] = v;
        else if (k < N + M) b[k - N] = v;
        else W[k - N - M] = v;
    }
}

/* ------------------------------------------------------------------------- */
/* Chain initialisation.  mode 0: sigma_i = +1 iff bit 0 of draw(i) word x0.  */
/* mode 1 (total S^z = 0, N even): start from N/2 up spins followed by N/2    */
/* down spins and apply a Fisher-Yates shuffle: for k = N-1 down to 1, swap   */
/* positions k and floor(x0*(k+1)/2^32) with x0 from draw(chain, k, tag 1).   */
/* ------------------------------------------------------------------------- */
void orc_init_chains(int N, int C, uint64_t seed, int mode, int8_t* spins) {
    for (int c = 0; c < C; ++c) {
        int8_t* s = spins + (long)c * N;
        if (mode == 0) {
            for (int i = 0; i < N; ++i) {
                uint32_t r[4];
                philox_draw(seed, (uint32_t)c, (uint64_t)i, 1u, r);
                s[i] = (r[0] & 1u) ? 1 : -1;
            }
        } else {
            for (int i = 0; i < N; ++i) s[i] = (i < N / 2) ? 1 : -1;
            for (int k = N - 1; k >= 1; --k) {
                uint32_t r[4];
                philox_draw(seed, (uint32_t)c, (uint64_t)k, 1u, r);
                int m = draw_index(r[0], k + 1);
                int8_t t = s[k]; s[k] = s[m]; s[m] = t;
            }
        }
    }
}

/* ------------------------------------------------------------------------- */
/* Lattice (Sec. VI): nearest-neighbour bonds with periodic boundaries.       */
/* kind 0 = chain of Lx sites: (i, i+1 mod N).                                */
/* kind 1 = Lx x Ly square: for every r, (r, r+x) then (r, r+y).              */
/* Bonds that coincide on a 2-wide lattice are kept twice.                    */
/* ------------------------------------------------------------------------- */
int orc_lattice_bonds(int kind, int Lx, int Ly, int* bonds) {
    int nb = 0;
    if (kind == 0) {
        for (int i = 0; i < Lx; ++i) { bonds[2 * nb] = i; bonds[2 * nb + 1] = (i + 1) % Lx; ++nb; }
    } else {
        for (int y = 0; y < Ly; ++y)
            for (int x = 0; x < Lx; ++x) {
                int r = x + Lx * y;
                bonds[2 * nb] = r; bonds[2 * nb + 1] = ((x + 1) % Lx) + Lx * y; ++nb;
                bonds[2 * nb] = r; bonds[2 * nb + 1] = x + Lx * ((y + 1) % Ly); ++nb;
            }
    }
    return nb;
}

/* ------------------------------------------------------------------------- */
/* RBM amplitude (Sec. I):                                                    */
/*   log psi(sigma) = sum_i a_i sigma_i + sum_j log(2 cosh theta_j),          */
/*   theta_j = b_j + sum_i W_ij sigma_i.                                      */
/* log(2cosh z) = s z + log(1 + exp(-2 s z)), s = sign(Re z): the principal   */
/* branch of the second term, so Im log psi is defined modulo 2 pi.           */
/* Near a zero of cosh, z = i pi (m + 1/2) + d with |d| small, 1 + exp(-2sz)  */
/* cancels to |d| and loses about log10(1/|d|) digits; there the identities   */
/* cosh z = i (-1)^m sinh d and tanh z = coth d are used instead, with        */
/* d = z - i pi (m + 1/2) formed with pi to about 32 digits (z itself is     */
/* exact: a sum of a few parameters).  Both forms are the definition; only    */
/* the rounding differs.                                                      */
/* ------------------------------------------------------------------------- */
/* pi = PI_HI + PI_LO to about 1e-32 (PI_HI the double nearest pi); the product PI_HI (m + 1/2) and its    */
/* exact rounding error (fma) keep d exact to about 1e-32 |m|.                                             */
static const double PI_LO = 1.2246467991473532e-16;

static int near_zero_of_cosh(cplx z, double* m, cplx* d) {
    *m = rint(cimag(z) / M_PI - 0.5);
    const double h = *m + 0.5, hi = M_PI * h, err = fma(M_PI, h, -hi);
    *d = creal(z) + I * (((cimag(z) - hi) - err) - PI_LO * h);
    return cabs(*d) < 0.5;
}

static cplx log2cosh(cplx z) {
    double m;
    cplx d;
    if (near_zero_of_cosh(z, &m, &d)) return log(2.0) + clog(csinh(d)) + I * (M_PI * (m + 0.5));
    double s = (creal(z) >= 0.0) ? 1.0 : -1.0;
    return s * z + clog(1.0 + cexp(-2.0 * s * z));
}

static cplx tanh_of(cplx z) {
    double m;
    cplx d;
    if (near_zero_of_cosh(z, &m, &d)) return ccosh(d) / csinh(d);
    return ctanh(z);
}

static void theta_of(int N, int M, const cplx* b, const cplx* W, const int8_t* sig, cplx* th) {
    for (int j = 0; j < M; ++j) th[j] = b[j];
    for (int i = 0; i < N; ++i) {
        double si = (double)sig[i];
        const cplx* Wi = W + (long)i * M;
        for (int j = 0; j < M; ++j) th[j] += si * Wi[j];
    }
}

static cplx logpsi_one(int N, int M, const cplx* a, const cplx* b, const cplx* W, const int8_t* sig, cplx* th) {
    theta_of(N, M, b, W, sig, th);
    cplx acc = 0.0;
    for (int i = 0; i < N; ++i) acc += a[i] * (double)sig[i];
    for (int j = 0; j < M; ++j) acc += log2cosh(th[j]);
    return acc;
}

void orc_logpsi(int N, int M, const cplx* a, const cplx* b, const cplx* W,
                const int8_t* sig, long n, cplx* out) {
#pragma omp parallel
    {
        cplx* th = (cplx*)malloc(sizeof(cplx) * (size_t)M);
#pragma omp for schedule(static)
        for (long s = 0; s < n; ++s) out[s] = logpsi_one(N, M, a, b, W, sig + s * N, th);
        free(th);
    }
}

/* Enumeration: sigma_i = +1 iff bit i of s is set, s = 0 .. 2^N - 1. */
void orc_enumerate(int N, int8_t* sig) {
    long n = 1L << N;
    for (long s = 0; s < n; ++s)
        for (int i = 0; i < N; ++i) sig[s * N + i] = ((s >> i) & 1L) ? 1 : -1;
}

/* Exact Born weights p(sigma) = |psi|^2 / sum |psi|^2 over all configurations. */
void orc_enum_weights(long n, const cplx* logpsi, double* p) {
    double mx = -INFINITY;
    for (long s = 0; s < n; ++s) if (2.0 * creal(logpsi[s]) > mx) mx = 2.0 * creal(logpsi[s]);
    double z = 0.0;
    for (long s = 0; s < n; ++s) { p[s] = exp(2.0 * creal(logpsi[s]) - mx); z += p[s]; }
    for (long s = 0; s < n; ++s) p[s] /= z;
}

/* f_q(sigma) = N^{-1/2} sum_r exp(-i q.r) sigma_r / 2: the momentum-space    */
/* S^z operator (App. B), diagonal in the S^z basis.                          */
static cplx fq_of(int kind, int Lx, int N, const double* q, const int8_t* sig) {
    cplx acc = 0.0;
    for (int r = 0; r < N; ++r) {
        int x = (kind == 0) ? r : r % Lx;
        int y = (kind == 0) ? 0 : r / Lx;
        double ph = q[0] * x + q[1] * y;
        acc += cexp(-I * ph) * (0.5 * (double)sig[r]);
    }
    return acc / sqrt((double)N);
}

void orc_fq(int kind, int Lx, int N, const double* q, const int8_t* sig, long n, cplx* out) {
    for (long s = 0; s < n; ++s) out[s] = fq_of(kind, Lx, N, q, sig + s * N);
}

/* ------------------------------------------------------------------------- */
/* Heisenberg local quantity (Sec. VI, H = J sum_<ij> S_i . S_j, with         */
/* S_i.S_j = S^z_i S^z_j + (S^+_i S^-_j + S^-_i S^+_j)/2):                    */
/*   (H g)(sigma) / g(sigma) = sum_bonds [ J/4 sigma_i sigma_j                */
/*        + [sigma_i != sigma_j] (J/2) g(sigma^{ij}) / g(sigma) ]             */
/* where g(sigma) = d(sigma) psi(sigma) with an optional diagonal factor d    */
/* (d = f_q makes g = t_0 = S^z_q psi), and sigma^{ij} swaps sites i and j.   */
/* Returned is (H g)(sigma) / psi(sigma), so that no division by d occurs.    */
/* ------------------------------------------------------------------------- */
static cplx hg_over_psi(int N, int M, const cplx* a, const cplx* b, const cplx* W,
                        int nb, const int* bonds, double J, const int8_t* sig,
                        int use_fq, int kind, int Lx, const double* q, int8_t* tmp, cplx* th) {
    cplx lp = logpsi_one(N, M, a, b, W, sig, th);
    cplx d0 = use_fq ? fq_of(kind, Lx, N, q, sig) : 1.0;
    cplx acc = 0.0;
    memcpy(tmp, sig, (size_t)N);
    for (int e = 0; e < nb; ++e) {
        int i = bonds[2 * e], j = bonds[2 * e + 1];
        acc += 0.25 * J * (double)(sig[i] * sig[j]) * d0;
        if (sig[i] != sig[j]) {
            tmp[i] = sig[j]; tmp[j] = sig[i];
            cplx lp2 = logpsi_one(N, M, a, b, W, tmp, th);
            cplx d1 = use_fq ? fq_of(kind, Lx, N, q, tmp) : 1.0;
            acc += 0.5 * J * d1 * cexp(lp2 - lp);
            tmp[i] = sig[i]; tmp[j] = sig[j];
        }
    }
    return acc;
}

/* E_loc(sigma) = (H psi)(sigma) / psi(sigma). */
void orc_local_energy(int N, int M, const cplx* a, const cplx* b, const cplx* W,
                      int kind, int Lx, int Ly, double J, const int8_t* sig, long n, cplx* out) {
    int* bonds = (int*)malloc(sizeof(int) * 4 * (size_t)N);
    int nb = orc_lattice_bonds(kind, Lx, Ly, bonds);
    double q0[2] = {0.0, 0.0};
#pragma omp parallel
    {
        int8_t* tmp = (int8_t*)malloc((size_t)N);
        cplx* th = (cplx*)malloc(sizeof(cplx) * (size_t)M);
#pragma omp for schedule(static)
        for (long s = 0; s < n; ++s)
            out[s] = hg_over_psi(N, M, a, b, W, nb, bonds, J, sig + s * N, 0, kind, Lx, q0, tmp, th);
        free(tmp); free(th);
    }
    free(bonds);
}

/* ------------------------------------------------------------------------- */
/* Log-derivatives (Sec. III, O_k = d psi / d alpha_k / psi; the RBM is       */
/* holomorphic in its parameters):                                            */
/*   O_{a_i} = sigma_i, O_{b_j} = tanh theta_j, O_{W_ij} = sigma_i tanh th_j. */
/* ------------------------------------------------------------------------- */
void orc_logderiv(int N, int M, const cplx* b, const cplx* W, const int8_t* sig, long n, cplx* O) {
    long P = (long)N + M + (long)N * M;
#pragma omp parallel
    {
        cplx* th = (cplx*)malloc(sizeof(cplx) * (size_t)M);
#pragma omp for schedule(static)
        for (long s = 0; s < n; ++s) {
            const int8_t* sg = sig + s * N;
            cplx* row = O + s * P;
            theta_of(N, M, b, W, sg, th);
            for (int i = 0; i < N; ++i) row[i] = (double)sg[i];
            for (int j = 0; j < M; ++j) row[N + j] = tanh_of(th[j]);
            for (int i = 0; i < N; ++i)
                for (int j = 0; j < M; ++j) row[N + M + (long)i * M + j] = (double)sg[i] * tanh_of(th[j]);
        }
        free(th);
    }
}

/* ------------------------------------------------------------------------- */
/* Chebyshev target ratio (Sec. III, recursion of the target states):         */
/* the state fitted at this stage is psi_{n+1} = t~_{n+1}; its target is      */
/*   order 0 : phi = beta_0 H~ t_0,             t_0 = f_q psi_gs              */
/*   order n>=1: phi = 2 beta_n H~ t~_n - beta_{n-1} t~_{n-1}                 */
/* with H~ = (H - E_c)/W_scale, t~_0 = t_0.  R(sigma) = phi(sigma) /          */
/* psi_{n+1}(sigma) is evaluated as exponentials of log-amplitude differences */
/* so that t_0(sigma) = 0 never appears in a denominator.                     */
/*   order 0 : psi_n = psi_gs (the factor f_q applied inside H~).             */
/*   order 1 : psi_nm1 = psi_gs, multiplied by f_q.                           */
/*   order>=2: psi_nm1 = t~_{n-1}.                                            */
/* hpsi_out receives (H g_n)(sigma) / psi_n(sigma), g_n = t_0 at order 0 and  */
/* psi_n otherwise (i.e. the local energy of psi_n for order >= 1).           */
/* ------------------------------------------------------------------------- */
typedef struct {
    int order;
    double E_c, W_scale;
    double beta_n[2], beta_nm1[2];
    double q[2];
} orc_cheb;

void orc_target_ratio(int N, int M,
                      const cplx* a1, const cplx* b1, const cplx* W1,      /* psi_{n+1} */
                      const cplx* an, const cplx* bn, const cplx* Wn,      /* psi_n */
                      const cplx* am, const cplx* bm, const cplx* Wm,      /* psi_{n-1} (may be NULL at order 0) */
                      const orc_cheb* ch, int kind, int Lx, int Ly, double J,
                      const int8_t* sig, long n, cplx* R, cplx* hpsi_out) {
    int* bonds = (int*)malloc(sizeof(int) * 4 * (size_t)N);
    int nb = orc_lattice_bonds(kind, Lx, Ly, bonds);
    cplx bn_c = ch->beta_n[0] + I * ch->beta_n[1];
    cplx bm_c = ch->beta_nm1[0] + I * ch->beta_nm1[1];
#pragma omp parallel
    {
        int8_t* tmp = (int8_t*)malloc((size_t)N);
        cplx* th = (cplx*)malloc(sizeof(cplx) * (size_t)M);
#pragma omp for schedule(static)
        for (long s = 0; s < n; ++s) {
            const int8_t* sg = sig + s * N;
            cplx l1 = logpsi_one(N, M, a1, b1, W1, sg, th);
            cplx ln = logpsi_one(N, M, an, bn, Wn, sg, th);
            int fq_n = (ch->order == 0);
            cplx hg = hg_over_psi(N, M, an, bn, Wn, nb, bonds, J, sg, fq_n, kind, Lx, ch->q, tmp, th);
            cplx dn = fq_n ? fq_of(kind, Lx, N, ch->q, sg) : 1.0;
            /* (H~ g_n)(sigma) / psi_n(sigma) */
            cplx ht = (hg - ch->E_c * dn) / ch->W_scale;
            cplx r;
            if (ch->order == 0) {
                r = bn_c * ht * cexp(ln - l1);
            } else {
                cplx lm = logpsi_one(N, M, am, bm, Wm, sg, th);
                cplx dm = (ch->order == 1) ? fq_of(kind, Lx, N, ch->q, sg) : 1.0;
                r = 2.0 * bn_c * ht * cexp(ln - l1) - bm_c * dm * cexp(lm - l1);
            }
            R[s] = r;
            if (hpsi_out) hpsi_out[s] = hg;
        }
        free(tmp); free(th);
    }
    free(bonds);
}

/* ------------------------------------------------------------------------- */
/* Metropolis sampling of P(s) = |psi_s|^2 / <psi|psi> (Sec. III).            */
/* Proposal at step t (t = step_offset + sweep*N + k), draw x = Philox(seed,  */
/* ctr = (chain, t, tag 0)): i = floor(x0 N / 2^32), j = floor(x1 N / 2^32),  */
/* u = (x2 >> 8) 2^-24.  proposal 0: flip site i.  proposal 1: swap sites i   */
/* and j when sigma_i != sigma_j, else a null move.  Accept iff               */
/* u < exp(2 Re[log psi(sigma') - log psi(sigma)]).  A sample is the state    */
/* after each sweep of N proposals.  Row c of spins is chain chain_ids[c]    */
/* (chain c when chain_ids is NULL): the chain index enters only the counter.  */
/*                                                                            */
/* Replay: if trace != NULL it holds one bit per proposal and chain (the      */
/* decisions of another implementation, bit t of word t/32 of the chain's     */
/* row of trace_words words).  Where the oracle's decision differs and        */
/* |u - r| <= margin * max(r, 1e-30) the step counts as ambiguous; a larger   */
/* gap counts as a mismatch.  Either way the traced decision is adopted, so   */
/* both trajectories stay aligned.                                            */
/* ------------------------------------------------------------------------- */
void orc_metropolis(int N, int M, const cplx* a, const cplx* b, const cplx* W,
                    int8_t* spins, int C, int n_sweeps, int proposal, uint64_t seed,
                    uint64_t step_offset, int8_t* samples_out, uint32_t* n_accept,
                    const uint32_t* trace, long trace_words, double margin,
                    long* n_ambiguous, long* n_mismatch, const int* chain_ids) {
    long amb = 0, mis = 0;
#pragma omp parallel reduction(+:amb, mis)
    {
        cplx* th = (cplx*)malloc(sizeof(cplx) * (size_t)M);
        int8_t* prop = (int8_t*)malloc((size_t)N);
#pragma omp for schedule(dynamic, 1)
        for (int c = 0; c < C; ++c) {
            int8_t* s = spins + (long)c * N;
            uint32_t acc = 0;
            for (int sw = 0; sw < n_sweeps; ++sw) {
                for (int k = 0; k < N; ++k) {
                    long tloc = (long)sw * N + k;
                    uint64_t t = step_offset + (uint64_t)tloc;
                    uint32_t r4[4];
                    philox_draw(seed, (uint32_t)(chain_ids ? chain_ids[c] : c), t, 0u, r4);
                    int i = draw_index(r4[0], N), j = draw_index(r4[1], N);
                    double u = draw_unit(r4[2]);
                    memcpy(prop, s, (size_t)N);
                    if (proposal == 0) {
                        prop[i] = (int8_t)(-s[i]);
                    } else {
                        if (s[i] == s[j]) continue;              /* null move */
                        prop[i] = s[j]; prop[j] = s[i];
                    }
                    cplx l0 = logpsi_one(N, M, a, b, W, s, th);
                    cplx l1 = logpsi_one(N, M, a, b, W, prop, th);
                    double r = exp(2.0 * creal(l1 - l0));
                    int dec = (u < r);
                    if (trace) {
                        int g = (int)((trace[(long)c * trace_words + tloc / 32] >> (tloc % 32)) & 1u);
                        if (g != dec) {
                            if (fabs(u - r) <= margin * fmax(r, 1e-30)) ++amb; else ++mis;
                            dec = g;
                        }
                    }
                    if (dec) { memcpy(s, prop, (size_t)N); ++acc; }
                }
                if (samples_out) memcpy(samples_out + ((long)sw * C + c) * N, s, (size_t)N);
            }
            if (n_accept) n_accept[c] = acc;
        }
        free(th); free(prop);
    }
    if (n_ambiguous) *n_ambiguous = amb;
    if (n_mismatch) *n_mismatch = mis;
}

/* ------------------------------------------------------------------------- */
/* Weighted FP64 sums (Kahan-compensated).                                    */
/* ------------------------------------------------------------------------- */
typedef struct { cplx s, c; } ksum;
static void kadd(ksum* k, cplx v) {
    cplx y = v - k->c;
    cplx t = k->s + y;
    k->c = (t - k->s) - y;
    k->s = t;
}

/* ------------------------------------------------------------------------- */
/* Hand-written Hermitian positive-definite solve A x = rhs by Cholesky       */
/* A = L L^H (A overwritten by L).  Returns 0, or -1 if a pivot is <= 0.      */
/* ------------------------------------------------------------------------- */
static int chol_solve(long P, cplx* A, cplx* x) {
    for (long j = 0; j < P; ++j) {
        double d = creal(A[j * P + j]);
        for (long k = 0; k < j; ++k) d -= creal(A[j * P + k] * conj(A[j * P + k]));
        if (!(d > 0.0)) return -1;
        double ljj = sqrt(d);
        A[j * P + j] = ljj;
        for (long i = j + 1; i < P; ++i) {
            cplx v = A[i * P + j];
            for (long k = 0; k < j; ++k) v -= A[i * P + k] * conj(A[j * P + k]);
            A[i * P + j] = v / ljj;
        }
    }
    for (long i = 0; i < P; ++i) {                 /* L y = rhs */
        cplx v = x[i];
        for (long k = 0; k < i; ++k) v -= A[i * P + k] * x[k];
        x[i] = v / creal(A[i * P + i]);
    }
    for (long i = P - 1; i >= 0; --i) {            /* L^H x = y */
        cplx v = x[i];
        for (long k = i + 1; k < P; ++k) v -= conj(A[k * P + i]) * x[k];
        x[i] = v / creal(A[i * P + i]);
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Natural-gradient (stochastic reconfiguration) step, Sec. III:              */
/*   gamma = arccos sqrt(|<R>|^2 / <|R|^2>),  beta = <R>,                     */
/*   F_k   = dgamma * gamma cot(gamma) * [ <O_k^* R>/<R> - <O_k^*> ],         */
/*   S_kk' = <O_k^* O_k'> - <O_k>^* <O_k'>,                                   */
/*   (S + eps I) dalpha = F,  alpha <- alpha + dalpha.                        */
/* <f> = sum_s w_s f_s with w_s = 1/n (weights == NULL) or the given weights. */
/* gamma cot gamma is replaced by 1 - gamma^2/3 for gamma < 1e-4.             */
/* stats: [gamma, Re beta, Im beta, |F|_2].  S_out / F_out / dalpha_out may   */
/* be NULL.  The parameters are updated in place.  Returns 0 or -1 if the     */
/* Cholesky factorisation fails.                                              */
/* ------------------------------------------------------------------------- */
int orc_sr_step(int N, int M, cplx* a, cplx* b, cplx* W, const int8_t* sig,
                const double* weights, const cplx* R, long n, double dgamma, double eps,
                double* stats, cplx* S_out, cplx* F_out, cplx* dalpha_out) {
    long P = (long)N + M + (long)N * M;
    cplx* O = (cplx*)malloc(sizeof(cplx) * (size_t)(n * P));
    orc_logderiv(N, M, b, W, sig, n, O);

    ksum kR = {0, 0};
    double r2 = 0.0, r2c = 0.0;
    for (long s = 0; s < n; ++s) {
        double w = weights ? weights[s] : 1.0 / (double)n;
        kadd(&kR, w * R[s]);
        double y = w * creal(R[s] * conj(R[s])) - r2c, t = r2 + y;
        r2c = (t - r2) - y; r2 = t;
    }
    cplx Rm = kR.s;
    double ratio = creal(Rm * conj(Rm)) / r2;
    double gamma = acos(fmin(1.0, sqrt(ratio)));
    double gcot = (gamma < 1e-4) ? 1.0 - gamma * gamma / 3.0 : gamma / tan(gamma);

    cplx* Om = (cplx*)calloc((size_t)P, sizeof(cplx));
    cplx* F = (cplx*)calloc((size_t)P, sizeof(cplx));
#pragma omp parallel for schedule(static)
    for (long k = 0; k < P; ++k) {
        ksum s1 = {0, 0}, s2 = {0, 0};
        for (long s = 0; s < n; ++s) {
            double w = weights ? weights[s] : 1.0 / (double)n;
            cplx o = O[s * P + k];
            kadd(&s1, w * o);
            kadd(&s2, w * conj(o) * R[s]);
        }
        Om[k] = s1.s;
        F[k] = dgamma * gcot * (s2.s / Rm - conj(s1.s));
    }

    cplx* S = (cplx*)malloc(sizeof(cplx) * (size_t)(P * P));
#pragma omp parallel for schedule(dynamic, 1)
    for (long k = 0; k < P; ++k) {
        for (long kp = 0; kp < P; ++kp) {
            ksum acc = {0, 0};
            for (long s = 0; s < n; ++s) {
                double w = weights ? weights[s] : 1.0 / (double)n;
                kadd(&acc, w * conj(O[s * P + k]) * O[s * P + kp]);
            }
            S[k * P + kp] = acc.s - conj(Om[k]) * Om[kp];
        }
    }
    if (S_out) memcpy(S_out, S, sizeof(cplx) * (size_t)(P * P));
    if (F_out) memcpy(F_out, F, sizeof(cplx) * (size_t)P);

    for (long k = 0; k < P; ++k) S[k * P + k] += eps;
    cplx* x = (cplx*)malloc(sizeof(cplx) * (size_t)P);
    memcpy(x, F, sizeof(cplx) * (size_t)P);
    int rc = chol_solve(P, S, x);
    if (rc == 0) {
        for (long k = 0; k < P; ++k) {
            if (k < N) a[k] += x[k];
            else if (k < N + M) b[k - N] += x[k];
            else W[k - N - M] += x[k];
        }
        if (dalpha_out) memcpy(dalpha_out, x, sizeof(cplx) * (size_t)P);
    }
    double fn = 0.0;
    for (long k = 0; k < P; ++k) fn += creal(F[k] * conj(F[k]));
    if (stats) { stats[0] = gamma; stats[1] = creal(Rm); stats[2] = cimag(Rm); stats[3] = sqrt(fn); }
    free(O); free(Om); free(F); free(S); free(x);
    return rc;
}

/* ------------------------------------------------------------------------- */
/* One log-derivative O_k(s) (Sec. III) from its definition: sigma_k for      */
/* k < N, tanh theta_j for the b rows, sigma_i tanh theta_j for W_ij.         */
/* ------------------------------------------------------------------------- */
static cplx logderiv_entry(int N, int M, const cplx* b, const cplx* W, const int8_t* sg, long k) {
    if (k < N) return (double)sg[k];
    const long r = k - N;
    const int j = (int)(r < M ? r : (r - M) % M);
    cplx th = b[j];
    for (int i = 0; i < N; ++i) th += (double)sg[i] * W[(long)i * M + j];
    const cplx t = tanh_of(th);
    if (r < M) return t;
    return (double)sg[(r - M) / M] * t;
}

/* ------------------------------------------------------------------------- */
/* The quantities of orc_sr_step restricted to the parameter indices          */
/* ks[0..nk): S_out[c][d] = S_{ks[c] ks[d]}, F_out[c] = F_{ks[c]},            */
/* Om_out[c] = <O_{ks[c]}>, stats = [gamma, Re beta, Im beta], every O_k(s)  */
/* formed per sample from its                                                  */
/* definition, so that models whose O [n][P] does not fit in memory can be    */
/* checked entry by entry.  The sample sums run over 64 fixed contiguous      */
/* blocks (compensated within a block) added in block order.                  */
/* ------------------------------------------------------------------------- */
void orc_sr_entries(int N, int M, const cplx* b, const cplx* W, const int8_t* sig,
                    const double* weights, const cplx* R, long n, double dgamma,
                    const long* ks, int nk, double* stats, cplx* S_out, cplx* F_out, cplx* Om_out) {
    ksum kR = {0, 0};
    double r2 = 0.0, r2c = 0.0;
    for (long s = 0; s < n; ++s) {
        double w = weights ? weights[s] : 1.0 / (double)n;
        kadd(&kR, w * R[s]);
        double y = w * creal(R[s] * conj(R[s])) - r2c, t = r2 + y;
        r2c = (t - r2) - y; r2 = t;
    }
    cplx Rm = kR.s;
    double gamma = acos(fmin(1.0, sqrt(creal(Rm * conj(Rm)) / r2)));
    double gcot = (gamma < 1e-4) ? 1.0 - gamma * gamma / 3.0 : gamma / tan(gamma);

    enum { NBLK = 64 };
    const long per = (n + NBLK - 1) / NBLK;
    const long stride = 2L * nk + (long)nk * nk;
    ksum* part = (ksum*)calloc((size_t)(NBLK * stride), sizeof(ksum));
#pragma omp parallel for schedule(dynamic, 1)
    for (int blk = 0; blk < NBLK; ++blk) {
        cplx* o = (cplx*)malloc(sizeof(cplx) * (size_t)nk);
        ksum* s1 = part + blk * stride;
        ksum* s2 = s1 + nk;
        ksum* g = s2 + nk;
        const long s0 = blk * per, s1e = (blk + 1) * per < n ? (blk + 1) * per : n;
        for (long s = s0; s < s1e; ++s) {
            const int8_t* sg = sig + s * N;
            double w = weights ? weights[s] : 1.0 / (double)n;
            for (int c = 0; c < nk; ++c) o[c] = logderiv_entry(N, M, b, W, sg, ks[c]);
            for (int c = 0; c < nk; ++c) {
                kadd(&s1[c], w * o[c]);
                kadd(&s2[c], w * conj(o[c]) * R[s]);
                for (int d = 0; d < nk; ++d) kadd(&g[(long)c * nk + d], w * conj(o[c]) * o[d]);
            }
        }
        free(o);
    }
    cplx* tot = (cplx*)calloc((size_t)stride, sizeof(cplx));
    for (long e = 0; e < stride; ++e) {
        ksum acc = {0, 0};
        for (int blk = 0; blk < NBLK; ++blk) kadd(&acc, part[blk * stride + e].s);
        tot[e] = acc.s;
    }
    const cplx* Om = tot;
    const cplx* ORm = tot + nk;
    const cplx* G = tot + 2 * nk;
    for (int c = 0; c < nk; ++c) {
        if (Om_out) Om_out[c] = Om[c];
        if (F_out) F_out[c] = dgamma * gcot * (ORm[c] / Rm - conj(Om[c]));
        if (S_out)
            for (int d = 0; d < nk; ++d) S_out[(long)c * nk + d] = G[(long)c * nk + d] - conj(Om[c]) * Om[d];
    }
    if (stats) { stats[0] = gamma; stats[1] = creal(Rm); stats[2] = cimag(Rm); }
    free(part); free(tot);
}

/* ------------------------------------------------------------------------- */
/* The diagonal of S and the means, for every parameter (Sec. III):           */
/*   S_kk = <|O_k|^2> - |<O_k>|^2,  Om_out[k] = <O_k>,  k in [0, P),          */
/* the full O row of each sample formed from its definition (as in           */
/* orc_logderiv) and summed as orc_sr_entries does: 64 fixed contiguous       */
/* blocks, compensated within a block, added in block order.  For models and  */
/* sample sets whose O [n][P] does not fit in memory.                         */
/* ------------------------------------------------------------------------- */
void orc_sr_diagonal(int N, int M, const cplx* b, const cplx* W, const int8_t* sig, const double* weights,
                     long n, double* S_out, cplx* Om_out) {
    const long P = (long)N + M + (long)N * M;
    enum { NBLK = 64 };
    const long per = (n + NBLK - 1) / NBLK;
    ksum* part = (ksum*)calloc((size_t)(NBLK * 2 * P), sizeof(ksum));
#pragma omp parallel for schedule(dynamic, 1)
    for (int blk = 0; blk < NBLK; ++blk) {
        cplx* th = (cplx*)malloc(sizeof(cplx) * (size_t)M);
        cplx* o = (cplx*)malloc(sizeof(cplx) * (size_t)P);
        ksum* s1 = part + (long)blk * 2 * P;
        ksum* s2 = s1 + P;
        const long s0 = blk * per, s1e = (blk + 1) * per < n ? (blk + 1) * per : n;
        for (long s = s0; s < s1e; ++s) {
            const int8_t* sg = sig + s * N;
            const double w = weights ? weights[s] : 1.0 / (double)n;
            theta_of(N, M, b, W, sg, th);
            for (int i = 0; i < N; ++i) o[i] = (double)sg[i];
            for (int j = 0; j < M; ++j) o[N + j] = tanh_of(th[j]);
            for (int i = 0; i < N; ++i)
                for (int j = 0; j < M; ++j) o[N + M + (long)i * M + j] = (double)sg[i] * o[N + j];
            for (long k = 0; k < P; ++k) {
                kadd(&s1[k], w * o[k]);
                kadd(&s2[k], w * creal(o[k] * conj(o[k])));
            }
        }
        free(th); free(o);
    }
    for (long k = 0; k < P; ++k) {
        ksum m = {0, 0}, q = {0, 0};
        for (int blk = 0; blk < NBLK; ++blk) {
            kadd(&m, part[(long)blk * 2 * P + k].s);
            kadd(&q, part[(long)blk * 2 * P + P + k].s);
        }
        if (Om_out) Om_out[k] = m.s;
        S_out[k] = creal(q.s) - creal(m.s * conj(m.s));
    }
    free(part);
}

/* ------------------------------------------------------------------------- */
/* Chebyshev moments (Sec. II; App. A for the momentum form), sampled over    */
/* s ~ |psi_gs|^2:                                                            */
/*   mu_0(q) = < |f_q|^2 >,                                                   */
/*   mu_n(q) = < f_q(s)^* beta_n t~_n(s) / psi_gs(s) >,  n = 1 .. n_max,      */
/* i.e. <t_0|t_n> / <psi_gs|psi_gs> with t_n ~ beta_n t~_n.                   */
/* t_params holds, for n = 1 .. n_max, the arrays a,b,W of t~_n packed as     */
/* [a(N) b(M) W(N*M)] consecutively; betas[n-1] = beta_n.                     */
/* mu_out is [n_q][n_max + 1].                                                */
/* ------------------------------------------------------------------------- */
void orc_moments(int N, int M, const cplx* ag, const cplx* bg, const cplx* Wg,
                 const cplx* t_params, const cplx* betas, int n_max,
                 const double* qs, int n_q, int kind, int Lx,
                 const int8_t* sig, const double* weights, long n, cplx* mu_out) {
    long P = (long)N + M + (long)N * M;
    cplx* lg = (cplx*)malloc(sizeof(cplx) * (size_t)n);
    orc_logpsi(N, M, ag, bg, Wg, sig, n, lg);
    cplx* B = (cplx*)malloc(sizeof(cplx) * (size_t)(n * (n_max + 1)));
    for (int t = 1; t <= n_max; ++t) {
        const cplx* tp = t_params + (long)(t - 1) * P;
        cplx* lt = (cplx*)malloc(sizeof(cplx) * (size_t)n);
        orc_logpsi(N, M, tp, tp + N, tp + N + M, sig, n, lt);
        for (long s = 0; s < n; ++s) B[s * (n_max + 1) + t] = betas[t - 1] * cexp(lt[s] - lg[s]);
        free(lt);
    }
    for (int iq = 0; iq < n_q; ++iq) {
        const double* q = qs + 2 * iq;
        ksum* acc = (ksum*)calloc((size_t)(n_max + 1), sizeof(ksum));
        for (long s = 0; s < n; ++s) {
            double w = weights ? weights[s] : 1.0 / (double)n;
            cplx f = fq_of(kind, Lx, N, q, sig + s * N);
            kadd(&acc[0], w * conj(f) * f);
            for (int t = 1; t <= n_max; ++t) kadd(&acc[t], w * conj(f) * B[s * (n_max + 1) + t]);
        }
        for (int t = 0; t <= n_max; ++t) mu_out[(long)iq * (n_max + 1) + t] = acc[t].s;
        free(acc);
    }
    free(lg); free(B);
}

/* ------------------------------------------------------------------------- */
/* Fidelity surrogate on a frozen sample set (drawn from |psi_{n+1}|^2):      */
/*   L(alpha) = (1/n) sum_s |1 - R(s; alpha)|^2,  R = phi / psi_{n+1}(alpha). */
/* Since R depends on alpha only through 1/psi_{n+1}, dR/dalpha_k = -R O_k    */
/* and dL/d conj(alpha_k) = (1/n) sum_s (1 - R_s) conj(R_s) conj(O_k(s)).     */
/* grad_out receives 2 dL/d conj(alpha) = dL/dRe alpha + i dL/dIm alpha.      */
/* R must be the target ratio at the current alpha.  Returns L.               */
/* ------------------------------------------------------------------------- */
double orc_fidelity_grad(int N, int M, const cplx* b, const cplx* W, const int8_t* sig,
                         const cplx* R, long n, cplx* grad_out) {
    long P = (long)N + M + (long)N * M;
    cplx* O = (cplx*)malloc(sizeof(cplx) * (size_t)(n * P));
    orc_logderiv(N, M, b, W, sig, n, O);
    double L = 0.0;
    for (long s = 0; s < n; ++s) { cplx d = 1.0 - R[s]; L += creal(d * conj(d)); }
    L /= (double)n;
    if (grad_out) {
#pragma omp parallel for schedule(static)
        for (long k = 0; k < P; ++k) {
            ksum acc = {0, 0};
            for (long s = 0; s < n; ++s)
                kadd(&acc, (1.0 - R[s]) * conj(R[s]) * conj(O[s * P + k]));
            grad_out[k] = 2.0 * acc.s / (double)n;
        }
    }
    free(O);
    return L;
}

/* The same gradient restricted to the parameter indices ks[0..nk), each      */
/* O_k(s) formed per sample (for models whose O [n][P] does not fit in        */
/* memory); sums over 64 fixed contiguous sample blocks added in block order.  */
/* Returns L.                                                                  */
double orc_fidelity_grad_entries(int N, int M, const cplx* b, const cplx* W, const int8_t* sig,
                                 const cplx* R, long n, const long* ks, int nk, cplx* grad_out) {
    double L = 0.0;
    for (long s = 0; s < n; ++s) { cplx d = 1.0 - R[s]; L += creal(d * conj(d)); }
    L /= (double)n;
    enum { NBLK = 64 };
    const long per = (n + NBLK - 1) / NBLK;
    ksum* part = (ksum*)calloc((size_t)(NBLK * nk), sizeof(ksum));
#pragma omp parallel for schedule(dynamic, 1)
    for (int blk = 0; blk < NBLK; ++blk) {
        const long s0 = blk * per, s1 = (blk + 1) * per < n ? (blk + 1) * per : n;
        for (long s = s0; s < s1; ++s) {
            const cplx c = (1.0 - R[s]) * conj(R[s]);
            for (int e = 0; e < nk; ++e)
                kadd(&part[blk * nk + e], c * conj(logderiv_entry(N, M, b, W, sig + s * N, ks[e])));
        }
    }
    for (int e = 0; e < nk; ++e) {
        ksum acc = {0, 0};
        for (int blk = 0; blk < NBLK; ++blk) kadd(&acc, part[blk * nk + e].s);
        grad_out[e] = 2.0 * acc.s / (double)n;
    }
    free(part);
    return L;
}

/* ------------------------------------------------------------------------- */
/* Batched moments over (q, n) instances (Sec. II moments, App. A momentum     */
/* form).  Instance i owns chains g in [offsets[i], offsets[i+1]) on psi_gs.  */
/* Chain g starts from the Fisher-Yates S^z = 0 configuration of              */
/* orc_init_chains (chain index g), runs n_burn + n_sweeps sweeps of the      */
/* orc_metropolis proposals (counter (g, t, tag 0), t = sweep*N + k), and     */
/* after each of the last n_sweeps sweeps adds |f_q(s)|^2 and                 */
/* conj(f_q(s)) beta_i t~_i(s)/psi_gs(s), every amplitude from scratch.       */
/* mu_out[i] = (<|f_q|^2>, <conj(f_q) beta t~/psi_gs>).  n_ambiguous counts   */
/* steps with |u - r| <= margin * max(r, 1e-30) (where a lower-precision      */
/* implementation could take the other branch).  With trace != NULL (row      */
/* g - offsets[0] of trace_words words per chain, the accept bits of another  */
/* implementation) the chains replay those decisions as orc_metropolis does: */
/* a differing decision counts as ambiguous within the margin, else as a     */
/* mismatch, and the traced one is adopted.                                   */
/* ------------------------------------------------------------------------- */
void orc_batched_moments(int N, int M, const cplx* ag, const cplx* bg, const cplx* Wg,
                         const cplx* t_params, const cplx* betas, const double* qs,
                         const int64_t* offsets, int n_inst, int n_burn, int n_sweeps, int proposal,
                         uint64_t seed, int kind, int Lx, double margin, cplx* mu_out, long* n_ambiguous,
                         const uint32_t* trace, long trace_words, long* n_mismatch) {
    long P = (long)N + M + (long)N * M;
    long amb = 0, mis = 0;
    for (int inst = 0; inst < n_inst; ++inst) {
        const cplx* tp = t_params + (long)inst * P;
        const double* q = qs + 2 * inst;
        const long n_ch = (long)(offsets[inst + 1] - offsets[inst]);
        /* per-chain sums, added in chain order below (the chains are independent) */
        cplx* c0 = (cplx*)calloc((size_t)(n_ch > 0 ? n_ch : 1), sizeof(cplx));
        cplx* c1 = (cplx*)calloc((size_t)(n_ch > 0 ? n_ch : 1), sizeof(cplx));
#pragma omp parallel for schedule(dynamic, 1) reduction(+:amb, mis)
        for (long c = 0; c < n_ch; ++c) {
            const int64_t g = offsets[inst] + c;
            const uint32_t* trow = trace ? trace + (long)(g - offsets[0]) * trace_words : NULL;
            int8_t* s = (int8_t*)malloc((size_t)N);
            int8_t* prop = (int8_t*)malloc((size_t)N);
            cplx* th = (cplx*)malloc(sizeof(cplx) * (size_t)M);
            ksum s0 = {0, 0}, s1 = {0, 0};
            for (int i = 0; i < N; ++i) s[i] = (i < N / 2) ? 1 : -1;
            for (int k = N - 1; k >= 1; --k) {
                uint32_t r[4];
                philox_draw(seed, (uint32_t)g, (uint64_t)k, 1u, r);
                int m = draw_index(r[0], k + 1);
                int8_t t = s[k]; s[k] = s[m]; s[m] = t;
            }
            for (int sw = 0; sw < n_burn + n_sweeps; ++sw) {
                for (int k = 0; k < N; ++k) {
                    uint32_t r4[4];
                    philox_draw(seed, (uint32_t)g, (uint64_t)sw * N + k, 0u, r4);
                    int i = draw_index(r4[0], N), j = draw_index(r4[1], N);
                    double u = draw_unit(r4[2]);
                    memcpy(prop, s, (size_t)N);
                    if (proposal == 0) prop[i] = (int8_t)(-s[i]);
                    else {
                        if (s[i] == s[j]) continue;
                        prop[i] = s[j]; prop[j] = s[i];
                    }
                    cplx l0 = logpsi_one(N, M, ag, bg, Wg, s, th);
                    cplx l1 = logpsi_one(N, M, ag, bg, Wg, prop, th);
                    double rr = exp(2.0 * creal(l1 - l0));
                    int dec = (u < rr);
                    if (trow) {
                        const long tloc = (long)sw * N + k;
                        const int gb = (int)((trow[tloc / 32] >> (tloc % 32)) & 1u);
                        if (gb != dec) {
                            if (fabs(u - rr) <= margin * fmax(rr, 1e-30)) ++amb; else ++mis;
                            dec = gb;
                        }
                    } else if (fabs(u - rr) <= margin * fmax(rr, 1e-30)) {
                        ++amb;
                    }
                    if (dec) memcpy(s, prop, (size_t)N);
                }
                if (sw < n_burn) continue;
                cplx f = fq_of(kind, Lx, N, q, s);
                cplx lg = logpsi_one(N, M, ag, bg, Wg, s, th);
                cplx lt = logpsi_one(N, M, tp, tp + N, tp + N + M, s, th);
                kadd(&s0, conj(f) * f);
                kadd(&s1, conj(f) * betas[inst] * cexp(lt - lg));
            }
            c0[c] = s0.s;
            c1[c] = s1.s;
            free(s); free(prop); free(th);
        }
        ksum t0 = {0, 0}, t1 = {0, 0};
        for (long c = 0; c < n_ch; ++c) { kadd(&t0, c0[c]); kadd(&t1, c1[c]); }
        const long cnt = n_ch * (long)n_sweeps;
        mu_out[2 * inst] = cnt ? t0.s / (double)cnt : 0.0;
        mu_out[2 * inst + 1] = cnt ? t1.s / (double)cnt : 0.0;
        free(c0); free(c1);
    }
    if (n_ambiguous) *n_ambiguous = amb;
    if (n_mismatch) *n_mismatch = mis;
}

/* ------------------------------------------------------------------------- */
/* Ground-state natural-gradient step (the paper obtains psi_gs by           */
/* minimising E = <psi|H psi>/<psi|psi> with Monte Carlo, Sec. I; the step   */
/* uses the same metric S as Sec. III):                                      */
/*   E = <E_loc>,  F_k = -lr [ <O_k^* E_loc> - <O_k>^* <E_loc> ]             */
/*     (the bracket is dE/d conj(alpha_k) for a holomorphic psi),            */
/*   (S + eps I) dalpha = F,  alpha <- alpha + dalpha.                        */
/* stats: [Re E, Im E, <|E_loc|^2> - |E|^2, |F|_2].  Returns 0 or -1.        */
/* ------------------------------------------------------------------------- */
int orc_sr_energy_step(int N, int M, cplx* a, cplx* b, cplx* W, const int8_t* sig,
                       const double* weights, const cplx* E, long n, double lr, double eps,
                       double* stats, cplx* S_out, cplx* F_out, cplx* dalpha_out) {
    long P = (long)N + M + (long)N * M;
    cplx* O = (cplx*)malloc(sizeof(cplx) * (size_t)(n * P));
    orc_logderiv(N, M, b, W, sig, n, O);
    ksum kE = {0, 0};
    double e2 = 0.0;
    for (long s = 0; s < n; ++s) {
        double w = weights ? weights[s] : 1.0 / (double)n;
        kadd(&kE, w * E[s]);
        e2 += w * creal(E[s] * conj(E[s]));
    }
    cplx Em = kE.s;
    cplx* Om = (cplx*)calloc((size_t)P, sizeof(cplx));
    cplx* F = (cplx*)calloc((size_t)P, sizeof(cplx));
#pragma omp parallel for schedule(static)
    for (long k = 0; k < P; ++k) {
        ksum s1 = {0, 0}, s2 = {0, 0};
        for (long s = 0; s < n; ++s) {
            double w = weights ? weights[s] : 1.0 / (double)n;
            cplx o = O[s * P + k];
            kadd(&s1, w * o);
            kadd(&s2, w * conj(o) * E[s]);
        }
        Om[k] = s1.s;
        F[k] = -lr * (s2.s - conj(s1.s) * Em);
    }
    cplx* S = (cplx*)malloc(sizeof(cplx) * (size_t)(P * P));
#pragma omp parallel for schedule(dynamic, 1)
    for (long k = 0; k < P; ++k)
        for (long kp = 0; kp < P; ++kp) {
            ksum acc = {0, 0};
            for (long s = 0; s < n; ++s) {
                double w = weights ? weights[s] : 1.0 / (double)n;
                kadd(&acc, w * conj(O[s * P + k]) * O[s * P + kp]);
            }
            S[k * P + kp] = acc.s - conj(Om[k]) * Om[kp];
        }
    if (S_out) memcpy(S_out, S, sizeof(cplx) * (size_t)(P * P));
    if (F_out) memcpy(F_out, F, sizeof(cplx) * (size_t)P);
    for (long k = 0; k < P; ++k) S[k * P + k] += eps;
    cplx* x = (cplx*)malloc(sizeof(cplx) * (size_t)P);
    memcpy(x, F, sizeof(cplx) * (size_t)P);
    int rc = chol_solve(P, S, x);
    if (rc == 0) {
        for (long k = 0; k < P; ++k) {
            if (k < N) a[k] += x[k];
            else if (k < N + M) b[k - N] += x[k];
            else W[k - N - M] += x[k];
        }
        if (dalpha_out) memcpy(dalpha_out, x, sizeof(cplx) * (size_t)P);
    }
    double fn = 0.0;
    for (long k = 0; k < P; ++k) fn += creal(F[k] * conj(F[k]));
    if (stats) {
        stats[0] = creal(Em); stats[1] = cimag(Em);
        stats[2] = e2 - creal(Em * conj(Em)); stats[3] = sqrt(fn);
    }
    free(O); free(Om); free(F); free(S); free(x);
    return rc;
}

/* ------------------------------------------------------------------------- */
/* Moment-correction matrices (Sec. IV; App. A, G and H) by sampling          */
/* s ~ |psi_gs|^2.  Basis vectors t_0 = S^z_q psi_gs and t_n = beta_n t~_n;   */
/* per sample B_n(s) = t_n(s)/psi_gs(s) and HB_n(s) = (H t_n)(s)/psi_gs(s):   */
/*   B_0 = f_q(s),  HB_0 from the Heisenberg action on f_q psi_gs;            */
/*   B_n = beta_n t~_n(s)/psi_gs(s),  HB_n = B_n (H t~_n)(s)/t~_n(s).         */
/*   G_nm = <conj(B_n) B_m>,  H_nm = <conj(B_n) HB_m>   (K = n_max + 1).      */
/* H is the physical Hamiltonian (units of J), not the rescaled one.          */
/* ------------------------------------------------------------------------- */
void orc_moment_matrices(int N, int M, const cplx* ag, const cplx* bg, const cplx* Wg,
                         const cplx* t_params, const cplx* betas, int n_max, const double* q,
                         int kind, int Lx, int Ly, double J, const int8_t* sig, const double* weights,
                         long n, cplx* G_out, cplx* H_out) {
    const long P = (long)N + M + (long)N * M;
    const int K = n_max + 1;
    int* bonds = (int*)malloc(sizeof(int) * 4 * (size_t)N);
    int nb = orc_lattice_bonds(kind, Lx, Ly, bonds);
    cplx* B = (cplx*)malloc(sizeof(cplx) * (size_t)(n * K));
    cplx* HB = (cplx*)malloc(sizeof(cplx) * (size_t)(n * K));
#pragma omp parallel
    {
        int8_t* tmp = (int8_t*)malloc((size_t)N);
        cplx* th = (cplx*)malloc(sizeof(cplx) * (size_t)M);
#pragma omp for schedule(static)
        for (long s = 0; s < n; ++s) {
            const int8_t* x = sig + s * N;
            const cplx lg = logpsi_one(N, M, ag, bg, Wg, x, th);
            B[s * K] = fq_of(kind, Lx, N, q, x);
            HB[s * K] = hg_over_psi(N, M, ag, bg, Wg, nb, bonds, J, x, 1, kind, Lx, q, tmp, th);
            for (int t = 1; t <= n_max; ++t) {
                const cplx* tp = t_params + (long)(t - 1) * P;
                const cplx lt = logpsi_one(N, M, tp, tp + N, tp + N + M, x, th);
                const cplx r = betas[t - 1] * cexp(lt - lg);
                const cplx el = hg_over_psi(N, M, tp, tp + N, tp + N + M, nb, bonds, J, x, 0, kind, Lx, q, tmp, th);
                B[s * K + t] = r;
                HB[s * K + t] = r * el;
            }
        }
        free(tmp); free(th);
    }
#pragma omp parallel for schedule(static)
    for (int e = 0; e < K * K; ++e) {
        const int k = e / K, l = e % K;
        ksum g = {0, 0}, h = {0, 0};
        for (long s = 0; s < n; ++s) {
            const double w = weights ? weights[s] : 1.0 / (double)n;
            kadd(&g, w * conj(B[s * K + k]) * B[s * K + l]);
            kadd(&h, w * conj(B[s * K + k]) * HB[s * K + l]);
        }
        G_out[e] = g.s;
        H_out[e] = h.s;
    }
    free(bonds); free(B); free(HB);
}

/* ------------------------------------------------------------------------- */
/* Symmetry-projected moment-correction matrices (App. A).                    */
/* The stored RBMs t_n00 approximate the Chebyshev vectors of the LOCAL       */
/* operator: t_000 = S^z_0 psi_gs (site 0 = origin) and t_n00 = beta_n t~_n.  */
/* A lattice symmetry g (a map of sites) acts on basis states so that         */
/* <s|g|t> = t(s o g) with (s o g)_r = s_{g(r)}.  With translations T_m and   */
/* the rotation R(x, y) = (L-1-y, x) of the L x L lattice,                     */
/*   B_{n,m,rot}(s) = <s|T_m R^rot|t_n00> / psi_gs(s),                         */
/* and the momentum-k projection of the rotation-averaged state is             */
/*   Bt_{nk}(s) = N^{-1/2} sum_m e^{-i k.m} (1/4) [B_{n,m,0} + B_{n,m+(1,0),1} */
/*                + B_{n,m+(1,1),2} + B_{n,m+(0,1),3}],   k.m = 2pi(k1 m1/Lx + k2 m2/Ly). */
/* On a chain (or with use_rot = 0) only the rot = 0 term is kept, with       */
/* weight 1.  HB uses (H t)(s o g) in place of t(s o g).  Then                */
/*   G^(k)_nn' = <conj(Bt_nk) Bt_n'k>,  H^(k)_nn' = <conj(Bt_nk) HBt_n'k>,     */
/* k = k1 + Lx k2 over all N momenta; G_out, H_out are [N][K][K].             */
/* ------------------------------------------------------------------------- */
static int sym_site(int kind, int Lx, int Ly, int m1, int m2, int rot, int r) {
    int x = (kind == 0) ? r : r % Lx, y = (kind == 0) ? 0 : r / Lx;
    for (int k = 0; k < rot; ++k) {         /* R(x, y) = (L-1-y, x), L = Lx = Ly */
        int nx = Lx - 1 - y, ny = x;
        x = nx; y = ny;
    }
    x = (x + m1) % Lx;
    y = (kind == 0) ? 0 : (y + m2) % Ly;
    return x + Lx * y;
}

/* sum over bonds of (H g)(y) / psi_ref with g(y) = f(y) exp(log t(y)), f = y_0/2 (local_f) or 1 */
static cplx h_apply_over(int N, int M, const cplx* a, const cplx* b, const cplx* W, int nb, const int* bonds,
                         double J, const int8_t* y, int local_f, cplx logref, int8_t* tmp, cplx* th) {
    const cplx ly = logpsi_one(N, M, a, b, W, y, th);
    const double fy = local_f ? 0.5 * (double)y[0] : 1.0;
    cplx acc = 0.0;
    memcpy(tmp, y, (size_t)N);
    for (int e = 0; e < nb; ++e) {
        const int i = bonds[2 * e], j = bonds[2 * e + 1];
        acc += 0.25 * J * (double)(y[i] * y[j]) * fy * cexp(ly - logref);
        if (y[i] != y[j]) {
            tmp[i] = y[j]; tmp[j] = y[i];
            const cplx l2 = logpsi_one(N, M, a, b, W, tmp, th);
            const double f2 = local_f ? 0.5 * (double)tmp[0] : 1.0;
            acc += 0.5 * J * f2 * cexp(l2 - logref);
            tmp[i] = y[i]; tmp[j] = y[j];
        }
    }
    return acc;
}

void orc_sym_matrices(int N, int M, const cplx* ag, const cplx* bg, const cplx* Wg,
                      const cplx* t_params, const cplx* betas, int n_max,
                      int kind, int Lx, int Ly, double J, int use_rot,
                      const int8_t* sig, const double* weights, long n, cplx* G_out, cplx* H_out) {
    const long P = (long)N + M + (long)N * M;
    const int K = n_max + 1;
    const int L2 = (kind == 0) ? 1 : Ly;
    const int nrot = (use_rot && kind == 1) ? 4 : 1;
    const int ng = N * nrot;                       /* group elements (m, rot) */
    int* bonds = (int*)malloc(sizeof(int) * 4 * (size_t)N);
    const int nb = orc_lattice_bonds(kind, Lx, Ly, bonds);
    /* per sample: Bt[s][k][t], HBt[s][k][t] */
    cplx* Bt = (cplx*)malloc(sizeof(cplx) * (size_t)n * N * K);
    cplx* HBt = (cplx*)malloc(sizeof(cplx) * (size_t)n * N * K);
#pragma omp parallel
    {
        int8_t* img = (int8_t*)malloc((size_t)N);
        int8_t* tmp = (int8_t*)malloc((size_t)N);
        cplx* th = (cplx*)malloc(sizeof(cplx) * (size_t)M);
        cplx* B = (cplx*)malloc(sizeof(cplx) * (size_t)K * ng);
        cplx* HB = (cplx*)malloc(sizeof(cplx) * (size_t)K * ng);
#pragma omp for schedule(dynamic, 4)
        for (long s = 0; s < n; ++s) {
            const int8_t* x = sig + s * N;
            const cplx lg = logpsi_one(N, M, ag, bg, Wg, x, th);
            for (int m2 = 0; m2 < L2; ++m2)
                for (int m1 = 0; m1 < Lx; ++m1)
                    for (int rot = 0; rot < nrot; ++rot) {
                        const int gi = ((m1 + Lx * m2) * nrot) + rot;
                        for (int r = 0; r < N; ++r) img[r] = x[sym_site(kind, Lx, Ly, m1, m2, rot, r)];
                        const cplx lgi = logpsi_one(N, M, ag, bg, Wg, img, th);
                        B[gi] = 0.5 * (double)img[0] * cexp(lgi - lg);
                        HB[gi] = h_apply_over(N, M, ag, bg, Wg, nb, bonds, J, img, 1, lg, tmp, th);
                        for (int t = 1; t <= n_max; ++t) {
                            const cplx* tp = t_params + (long)(t - 1) * P;
                            const cplx lt = logpsi_one(N, M, tp, tp + N, tp + N + M, img, th);
                            B[(long)t * ng + gi] = betas[t - 1] * cexp(lt - lg);
                            HB[(long)t * ng + gi] = betas[t - 1] *
                                h_apply_over(N, M, tp, tp + N, tp + N + M, nb, bonds, J, img, 0, lg, tmp, th);
                        }
                    }
            /* the App. A combination for every momentum */
            const int off[4][2] = {{0, 0}, {1, 0}, {1, 1}, {0, 1}};
            for (int k2 = 0; k2 < L2; ++k2)
                for (int k1 = 0; k1 < Lx; ++k1) {
                    const int kk = k1 + Lx * k2;
                    for (int t = 0; t < K; ++t) {
                        cplx sb = 0.0, sh = 0.0;
                        for (int m2 = 0; m2 < L2; ++m2)
                            for (int m1 = 0; m1 < Lx; ++m1) {
                                const double ph = 2.0 * M_PI * ((double)(k1 * m1) / Lx + (double)(k2 * m2) / Ly);
                                const cplx e = cexp(-I * ph);
                                cplx vb = 0.0, vh = 0.0;
                                for (int rot = 0; rot < nrot; ++rot) {
                                    const int a1 = (m1 + off[rot][0]) % Lx;
                                    const int a2 = (kind == 0) ? 0 : (m2 + off[rot][1]) % Ly;
                                    const int gi = ((a1 + Lx * a2) * nrot) + rot;
                                    vb += B[(long)t * ng + gi];
                                    vh += HB[(long)t * ng + gi];
                                }
                                sb += e * vb / (double)nrot;
                                sh += e * vh / (double)nrot;
                            }
                        Bt[((long)s * N + kk) * K + t] = sb / sqrt((double)N);
                        HBt[((long)s * N + kk) * K + t] = sh / sqrt((double)N);
                    }
                }
        }
        free(img); free(tmp); free(th); free(B); free(HB);
    }
    /* G^(k)_tu and H^(k)_tu summed in sample order */
#pragma omp parallel for schedule(static)
    for (long e = 0; e < (long)N * K * K; ++e) {
        const int kk = (int)(e / ((long)K * K)), t = (int)((e / K) % K), u = (int)(e % K);
        ksum g = {0, 0}, h = {0, 0};
        for (long s = 0; s < n; ++s) {
            const double w = weights ? weights[s] : 1.0 / (double)n;
            const cplx bt = conj(Bt[((long)s * N + kk) * K + t]);
            kadd(&g, w * bt * Bt[((long)s * N + kk) * K + u]);
            kadd(&h, w * bt * HBt[((long)s * N + kk) * K + u]);
        }
        G_out[e] = g.s;
        H_out[e] = h.s;
    }
    free(bonds); free(Bt); free(HBt);
}
