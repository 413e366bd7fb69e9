// Batched Chebyshev moments: many (q, n) instances in one persistent launch.
//
// Instance i pairs a momentum q_i with a stored Chebyshev state t~_i and its
// beta_i (Sec. III); its moment is mu_i = < f_{q_i}(s)^* beta_i t~_i(s)/psi_gs(s) >
// over s ~ |psi_gs|^2 (Sec. II, App. A), and mu0_i = < |f_{q_i}(s)|^2 >.
// Every instance owns its own number of Markov chains on psi_gs.  A chain is
// the unit of work: waves of a persistent grid take chains from an atomic
// counter until all are done, so uneven chain counts per instance do not
// unbalance the launch.  Per chain the wave keeps theta of psi_gs (for the
// acceptance) and theta of t~_i (for the ratio) in registers and updates both
// on every accepted exchange; after each recorded sweep it adds the chain's
// terms in double precision.  Per-chain partial sums are reduced per instance
// in chain order by a second kernel, so the result does not depend on the
// schedule.  All launches are stream-ordered kernels (no host work), so the
// sequence can be captured in a graph.
#include <hip/hip_runtime.h>

#include "device.hpp"
#include "internal.hpp"

namespace crbm {



__global__ void k_batched_reset(unsigned long long* counter) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *counter = 0ull;
}

template <int E>
__global__ __launch_bounds__(512) void k_batched(BatchedArgs A) {
    extern __shared__ int8_t s_spins[];           // one 256-byte row per wave
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    int8_t* row = s_spins + wv * 256;
    const int N = A.N, M = A.M;
    for (;;) {
        unsigned long long g = 0;
        if (lane == 0) g = atomicAdd(A.counter, 1ull);
        g = (unsigned long long)__builtin_amdgcn_readfirstlane((int)(g & 0xFFFFFFFFull)) |
            ((unsigned long long)__builtin_amdgcn_readfirstlane((int)(g >> 32)) << 32);
        if ((int64_t)g >= A.total) break;
        // instance of chain g: largest i with offsets[i] <= g
        int lo = 0, hi = A.n_inst;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (A.offsets[mid] <= (int64_t)g) lo = mid; else hi = mid;
        }
        const int inst = uniform(lo);
        const float2* tp = A.t_params + (long)inst * A.P;
        const float2* at = tp;
        const float2* bt = tp + N;
        const float2* Wt = tp + N + M;
        const double q0 = A.q[2 * inst], q1 = A.q[2 * inst + 1];

        // Fisher-Yates start at total S^z = 0 (Philox tag 1, counter a = chain id)
        if (lane == 0) {
            for (int i = 0; i < N; ++i) row[i] = (i < N / 2) ? 1 : -1;
            for (int k = N - 1; k >= 1; --k) {
                const int m = draw_index(draw(A.seed, (uint32_t)g, (uint64_t)k, 1u).x, k + 1);
                const int8_t t = row[k];
                row[k] = row[m];
                row[m] = t;
            }
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        WaveSpins sp;
        sp.load(row, N, lane);

        // theta of psi_gs and of t~_inst from the spins; the phases of this lane's sites
        float2 thg[E], tht[E];
        float Lg[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int k = e * kWave + lane;
            thg[e] = (k < M) ? A.gs.b[k] : make_float2(0.f, 0.f);
            tht[e] = (k < M) ? bt[k] : make_float2(0.f, 0.f);
        }
        for (int i = 0; i < N; ++i) {
            const float si = (float)sp.get(i);
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int k = e * kWave + lane;
                if (k < M) {
                    const float2 wg = A.gs.W[(long)i * M + k], wt = Wt[(long)i * M + k];
                    thg[e].x = fmaf(si, wg.x, thg[e].x);
                    thg[e].y = fmaf(si, wg.y, thg[e].y);
                    tht[e].x = fmaf(si, wt.x, tht[e].x);
                    tht[e].y = fmaf(si, wt.y, tht[e].y);
                }
            }
        }
#pragma unroll
        for (int e = 0; e < E; ++e) Lg[e] = (e * kWave + lane < M) ? re_log2cosh_fast(thg[e]) : 0.f;
        float2 ph[4];
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) {
            const int site = qq * kWave + lane;
            ph[qq] = make_float2(0.f, 0.f);
            if (site < N) {
                const int x = A.kind == 0 ? site : site % A.Lx;
                const int y = A.kind == 0 ? 0 : site / A.Lx;
                double sn, cs;
                sincos(q0 * x + q1 * y, &sn, &cs);
                ph[qq] = make_float2((float)cs, (float)-sn);
            }
        }
        const double2 beta = A.betas[inst];
        double m0 = 0.0, mr = 0.0, mi = 0.0;
        const int total_sweeps = A.n_burn + A.n_sweeps;
        uint32_t tw = 0;                          // accept bits of the current trace word
        uint32_t* trow = A.trace ? A.trace + (long)g * A.trace_words : nullptr;
        for (int sw = 0; sw < total_sweeps; ++sw) {
            for (int p = 0; p < N; ++p) {
                const uint64_t t = (uint64_t)sw * N + p;
                if (trow && t > 0 && (t & 31) == 0) {
                    if (lane == 0) trow[(t - 1) >> 5] = tw;
                    tw = 0;
                }
                const u32x4 x = draw(A.seed, (uint32_t)g, t, 0u);
                const int i = uniform(draw_index(x.x, N));
                const int j = uniform(draw_index(x.y, N));
                const float u = draw_unit(x.z);
                const int si = sp.get(i), sj = sp.get(j);
                const bool pair = A.proposal == 1;
                if (pair && si == sj) continue;
                const float m2si = -2.f * (float)si;
                float2 tn[E];
                float Ln[E];
                float dsum = 0.f;
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const int k = e * kWave + lane;
                    if (k < M) {
                        float2 d = A.gs.W[(long)i * M + k];
                        if (pair) d = csub(d, A.gs.W[(long)j * M + k]);
                        tn[e].x = fmaf(m2si, d.x, thg[e].x);
                        tn[e].y = fmaf(m2si, d.y, thg[e].y);
                        Ln[e] = re_log2cosh_fast(tn[e]);
                        dsum += Ln[e] - Lg[e];
                    } else {
                        tn[e] = thg[e];
                        Ln[e] = Lg[e];
                    }
                }
                float dl = uniform(wave_sum(dsum));
                float da = m2si * A.gs.a[i].x;
                if (pair) da -= m2si * A.gs.a[j].x;
                dl += da;
                if (u < __expf(2.f * dl)) {
                    tw |= 1u << (t & 31);
#pragma unroll
                    for (int e = 0; e < E; ++e) {
                        const int k = e * kWave + lane;
                        thg[e] = tn[e];
                        Lg[e] = Ln[e];
                        if (k < M) {
                            float2 d = Wt[(long)i * M + k];
                            if (pair) d = csub(d, Wt[(long)j * M + k]);
                            tht[e].x = fmaf(m2si, d.x, tht[e].x);
                            tht[e].y = fmaf(m2si, d.y, tht[e].y);
                        }
                    }
                    sp.set(i, -si, lane);
                    if (pair) sp.set(j, -sj, lane);
                }
            }
            if (sw < A.n_burn) continue;
            // f_q(s), and the ratio t~(s)/psi_gs(s) summed element by element
            float2 f = make_float2(0.f, 0.f), dlog = make_float2(0.f, 0.f);
#pragma unroll
            for (int qq = 0; qq < 4; ++qq) {
                const int site = qq * kWave + lane;
                if (site < N) {
                    const float s = (float)sp.s[qq];
                    f = cadd(f, cscale(ph[qq], 0.5f * s));
                    dlog = cadd(dlog, cscale(csub(at[site], A.gs.a[site]), s));
                }
            }
#pragma unroll
            for (int e = 0; e < E; ++e)
                if (e * kWave + lane < M) dlog = cadd(dlog, csub(log2cosh(tht[e]), log2cosh(thg[e])));
            f = wave_sum(f);
            dlog = wave_sum(dlog);
            const float2 r = cexpf(dlog);
            const double fx = (double)f.x * (1.0 / sqrt((double)N)), fy = (double)f.y * (1.0 / sqrt((double)N));
            const double2 br = zmul(beta, make_double2((double)r.x, (double)r.y));
            m0 += fx * fx + fy * fy;
            mr += fx * br.x + fy * br.y;          // conj(f) * (beta r)
            mi += fx * br.y - fy * br.x;
        }
        if (lane == 0) {
            A.partial[2 * g] = make_double2(m0, 0.0);
            A.partial[2 * g + 1] = make_double2(mr, mi);
            if (trow) trow[((uint64_t)total_sweeps * N - 1) >> 5] = tw;
        }
    }
}

// mu_out[i] = (sum of chain partials of instance i) / (c_i n_sweeps)
__global__ void k_batched_reduce(const double2* __restrict__ partial, const int64_t* __restrict__ offsets, int n_inst,
                                 int n_sweeps, double2* __restrict__ mu) {
    const int i = blockIdx.x;
    if (i >= n_inst) return;
    __shared__ double sh[4][4];
    const int64_t b = offsets[i], e = offsets[i + 1];
    double a0 = 0, ar = 0, ai = 0;
    for (int64_t c = b + threadIdx.x; c < e; c += blockDim.x) {
        a0 += partial[2 * c].x;
        ar += partial[2 * c + 1].x;
        ai += partial[2 * c + 1].y;
    }
    a0 = wave_sum(a0); ar = wave_sum(ar); ai = wave_sum(ai);
    if ((threadIdx.x & 63) == 0) { sh[0][threadIdx.x >> 6] = a0; sh[1][threadIdx.x >> 6] = ar; sh[2][threadIdx.x >> 6] = ai; }
    __syncthreads();
    if (threadIdx.x == 0) {
        const double cnt = (double)(e - b) * (double)n_sweeps;
        const double inv = cnt > 0 ? 1.0 / cnt : 0.0;
        mu[2 * i] = make_double2((sh[0][0] + sh[0][1] + sh[0][2] + sh[0][3]) * inv, 0.0);
        mu[2 * i + 1] = make_double2((sh[1][0] + sh[1][1] + sh[1][2] + sh[1][3]) * inv,
                                     (sh[2][0] + sh[2][1] + sh[2][2] + sh[2][3]) * inv);
    }
}

hipError_t launch_batched(const BatchedArgs& A, int blocks, int waves_per_block, double2* mu, hipStream_t stream) {
    hipLaunchKernelGGL(k_batched_reset, dim3(1), dim3(64), 0, stream, A.counter);
    const int E = (A.M + kWave - 1) / kWave;
    const dim3 grid(blocks), block(64 * waves_per_block);
    const size_t lds = 256 * (size_t)waves_per_block;
    switch (E) {
#define CRBM_CASE(e) case e: hipLaunchKernelGGL(k_batched<e>, grid, block, lds, stream, A); break;
        CRBM_CASE(1) CRBM_CASE(2) CRBM_CASE(3) CRBM_CASE(4) CRBM_CASE(5) CRBM_CASE(6) CRBM_CASE(7) CRBM_CASE(8)
#undef CRBM_CASE
        default: return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL(k_batched_reduce, dim3(A.n_inst), dim3(256), 0, stream, A.partial, A.offsets, A.n_inst,
                       A.n_sweeps, mu);
    return hipGetLastError();
}

}  // namespace crbm
