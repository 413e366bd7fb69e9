// Parameter initialisation, chain initialisation and the Metropolis sweep.
//
// Sampling (Sec. III): configurations s are drawn from |psi_s|^2 / <psi|psi>
// by Metropolis chains.  One wavefront owns one chain: lane l keeps the
// hidden units k = 64 e + l (e < E) of theta in registers together with the
// cached Re log(2 cosh theta_k), and the spins of sites 64 q + l.  A proposal
// touches rows W_i (and W_j), recomputes Re log(2 cosh theta'_k) per element,
// reduces the change over the wave and accepts on u < |psi'/psi|^2; only the
// real part of the log-amplitude is needed for the acceptance, so the
// imaginary part (and its atan2) never enters the inner loop.  theta is
// rebuilt from the spins at the start of every call.
#include "device.hpp"
#include "internal.hpp"
#include "sweep.hpp"

namespace crbm {

// ------------------------------------------------------------------ init_rbm
__global__ void k_init_rbm(float2* __restrict__ a, float2* __restrict__ b, float2* __restrict__ W, int N, int M,
                           uint64_t seed, float stddev) {
    const long P = (long)N + M + (long)N * M;
    const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= P) return;
    const u32x4 r = draw(seed, (uint32_t)k, 0ull, 2u);
    const float u1 = ((float)(r.x >> 8) + 1.0f) * (1.0f / 16777216.0f);
    const float u2 = (float)(r.y >> 8) * (1.0f / 16777216.0f);
    const float rad = stddev * sqrtf(-2.0f * logf(u1));
    float sn, cs;
    sincospif(2.0f * u2, &sn, &cs);
    const float2 v = make_float2(rad * cs, rad * sn);
    if (k < N) a[k] = v;
    else if (k < N + M) b[k - N] = v;
    else W[k - N - M] = v;
}

hipError_t launch_init_rbm(float2* a, float2* b, float2* W, int N, int M, uint64_t seed, float stddev,
                           hipStream_t stream) {
    const long P = (long)N + M + (long)N * M;
    const int threads = 256;
    const long blocks = (P + threads - 1) / threads;
    hipLaunchKernelGGL(k_init_rbm, dim3((unsigned)blocks), dim3(threads), 0, stream, a, b, W, N, M, seed, stddev);
    return hipGetLastError();
}

// ------------------------------------------------------------------ init_chains
// One thread per chain; the configuration is built in LDS (N <= 256).
__global__ __launch_bounds__(64) void k_init_chains(int8_t* __restrict__ spins, int N, int n_chains, uint64_t seed,
                                                    int zero_mag) {
    __shared__ int8_t buf[64][256];
    const int c = blockIdx.x * 64 + threadIdx.x;
    if (c >= n_chains) return;
    int8_t* s = buf[threadIdx.x];
    if (!zero_mag) {
        for (int i = 0; i < N; ++i) s[i] = (draw(seed, (uint32_t)c, (uint64_t)i, 1u).x & 1u) ? 1 : -1;
    } else {
        for (int i = 0; i < N; ++i) s[i] = (i < N / 2) ? 1 : -1;
        for (int k = N - 1; k >= 1; --k) {
            const int m = draw_index(draw(seed, (uint32_t)c, (uint64_t)k, 1u).x, k + 1);
            const int8_t t = s[k];
            s[k] = s[m];
            s[m] = t;
        }
    }
    for (int i = 0; i < N; ++i) spins[(long)c * N + i] = s[i];
}

hipError_t launch_init_chains(int8_t* spins, int N, int n_chains, uint64_t seed, int zero_mag, hipStream_t stream) {
    const int blocks = (n_chains + 63) / 64;
    hipLaunchKernelGGL(k_init_chains, dim3(blocks), dim3(64), 0, stream, spins, N, n_chains, seed, zero_mag);
    return hipGetLastError();
}

// ------------------------------------------------------------------ Metropolis sweep
// Rows are read only for live moves (an exchange of equal spins changes nothing), and all loads of a
// move are issued together before the first use.
struct SweepPos {
    long tloc;   // proposal index within this call
    int p, sw;   // position within the sweep, sweep index
};

// One proposal: a single flip, or with PAIR an exchange of sites i and j.
template <int E, bool PAIR>
__device__ __forceinline__ void sweep_step(const SampleArgs& A, int chain, int lane, SweepPos& pos,
                                           WaveSpins& sp, float2 (&th)[E], float (&L)[E], uint32_t& accepted,
                                           uint32_t& bits, DrawBatch& batch) {
    const int M = A.M;
    Proposal cur = next_proposal(batch, A.seed, (uint32_t)chain, A.step_offset, pos.tloc, lane, A.N);
    const int si = sp.get(cur.i);
    const int sj = sp.get(cur.j);
    if (!(PAIR && si == sj)) {
        float2 wi[E], wj[E], tn[E];
        float Ln[E];
        fetch_rows<E, PAIR>(A.psi, M, cur, lane, wi, wj);
        const float dl = proposal_dlog<E, PAIR>(cur, si, wi, wj, th, L, tn, Ln, lane, M);
        if (cur.u < __expf(2.f * dl)) {
#pragma unroll
            for (int e = 0; e < E; ++e) { th[e] = tn[e]; L[e] = Ln[e]; }
            sp.set(cur.i, -si, lane);
            if (PAIR) sp.set(cur.j, -sj, lane);
            ++accepted;
            bits |= 1u << (pos.tloc & 31);
        }
    }
    if (A.trace && ((pos.tloc & 31) == 31)) {
        if (lane == 0) A.trace[(long)chain * A.trace_words + (pos.tloc >> 5)] = bits;
        bits = 0;
    }
    ++pos.tloc;
    if (++pos.p == A.N) {
        if (A.samples_out) sp.store(A.samples_out + ((long)pos.sw * A.n_chains + chain) * A.N, A.N, lane);
        pos.p = 0;
        ++pos.sw;
    }
}

template <int E, bool PAIR>
__global__ __launch_bounds__(256) void k_sample(SampleArgs A) {
    const int lane = threadIdx.x & 63;
    const int chain = uniform((int)(blockIdx.x * 4 + (threadIdx.x >> 6)));
    if (chain >= A.n_chains) return;
    const int N = A.N, M = A.M;
    const float2* __restrict__ W = A.psi.W;
    const float2* __restrict__ av = A.psi.a;

    WaveSpins sp;
    sp.load(A.spins + (long)chain * N, N, lane);

    // theta = b + sigma W; lanes past M keep theta = 0, and their cached L is
    // the same function of the same value, so they add exactly zero below
    float2 th[E];
    float L[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int k = e * kWave + lane;
        th[e] = (k < M) ? A.psi.b[k] : make_float2(0.f, 0.f);
    }
#pragma unroll 4
    for (int i = 0; i < N; ++i) {
        const float si = (float)sp.get(i);
        const float2* Wi = W + (long)i * M;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int k = e * kWave + lane;
            const float2 w = Wi[min(k, M - 1)];
            const float s = (k < M) ? si : 0.f;
            th[e].x = fmaf(s, w.x, th[e].x);
            th[e].y = fmaf(s, w.y, th[e].y);
        }
    }
#pragma unroll
    for (int e = 0; e < E; ++e) L[e] = re_log2cosh_fast(th[e]);

    uint32_t accepted = 0, bits = 0;
    const long total = (long)A.n_sweeps * N;
    SweepPos pos{0, 0, 0};
    DrawBatch batch;
    while (pos.tloc < total) sweep_step<E, PAIR>(A, chain, lane, pos, sp, th, L, accepted, bits, batch);
    if (A.trace && (total & 31) != 0 && lane == 0) A.trace[(long)chain * A.trace_words + (total >> 5)] = bits;

    sp.store(A.spins + (long)chain * N, N, lane);
    if (A.n_accept && lane == 0) A.n_accept[chain] = accepted;
    if (A.theta_out) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int k = e * kWave + lane;
            if (k < M) A.theta_out[(long)chain * M + k] = th[e];
        }
    }
    if (A.logpsi_out) {
        // full complex log psi of the final state
        float2 acc = make_float2(0.f, 0.f);
#pragma unroll
        for (int e = 0; e < E; ++e)
            if (e * kWave + lane < M) acc = cadd(acc, log2cosh(th[e]));
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int site = q * kWave + lane;
            if (site < N) acc = cadd(acc, cscale(av[site], (float)sp.s[q]));
        }
        acc = wave_sum(acc);
        if (lane == 0) A.logpsi_out[chain] = acc;
    }
}

hipError_t launch_sample(const SampleArgs& args, hipStream_t stream) {
    const int E = (args.M + kWave - 1) / kWave;
    const dim3 grid((args.n_chains + 3) / 4), block(256);
    const bool pair = args.proposal == 1;
    switch (E) {
#define CRBM_CASE(e)                                                                                   \
    case e:                                                                                            \
        if (pair) hipLaunchKernelGGL((k_sample<e, true>), grid, block, 0, stream, args);               \
        else hipLaunchKernelGGL((k_sample<e, false>), grid, block, 0, stream, args);                   \
        break;
        CRBM_CASE(1) CRBM_CASE(2) CRBM_CASE(3) CRBM_CASE(4) CRBM_CASE(5) CRBM_CASE(6) CRBM_CASE(7) CRBM_CASE(8)
#undef CRBM_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace crbm
