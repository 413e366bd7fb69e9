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
// on every accepted move (theta of t~_i at the next accepted move or
// measurement, so that its row reads overlap the proposals in between); after
// each recorded sweep it adds the chain's terms in double precision.  The rows
// of psi_gs, the same for every chain, are read from a copy in LDS when it fits
// without lowering the occupancy: every live proposal reads two of them, and
// from L2 those reads, with the rows of t~_i, ran at the L2 gather ceiling.  Per-chain partial sums are reduced per instance
// in chain order by a second kernel, so the result does not depend on the
// schedule.  All launches are stream-ordered kernels (no host work), so the
// sequence can be captured in a graph.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "../../include/chebrbm.h"
#include "device.hpp"
#include "internal.hpp"
#include "sweep.hpp"

namespace crbm {

// LDS of one compute unit (gfx950), the most one block of k_batched may ask for
constexpr int kMaxBatchedLds = 160 * 1024;
constexpr int kMaxDevices = 64;

__global__ void k_batched_reset(unsigned long long* counter) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *counter = 0ull;
}

__global__ void k_clear_u64(unsigned long long* p, long n) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) p[e] = 0ull;
}

hipError_t launch_clear_u64(unsigned long long* p, long n, hipStream_t stream) {
    hipLaunchKernelGGL(k_clear_u64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, p, n);
    return hipGetLastError();
}

// Value at site i (wave-uniform) of a per-lane array holding sites 64 q + lane; ONE: all sites in slot 0
// (N <= 64), a single readlane.
template <bool ONE, typename T>
__device__ __forceinline__ T site_value(const T (&v)[4], int i) {
    const int l = i & 63;
    if (ONE) return __builtin_bit_cast(T, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v[0]), l));
    const int q = i >> 6;
    const int v0 = __builtin_amdgcn_readlane(__builtin_bit_cast(int, v[0]), l);
    const int v1 = __builtin_amdgcn_readlane(__builtin_bit_cast(int, v[1]), l);
    const int v2 = __builtin_amdgcn_readlane(__builtin_bit_cast(int, v[2]), l);
    const int v3 = __builtin_amdgcn_readlane(__builtin_bit_cast(int, v[3]), l);
    return __builtin_bit_cast(T, q == 0 ? v0 : q == 1 ? v1 : q == 2 ? v2 : v3);
}

// Spins of a chain of N <= 64 sites as one wave-uniform 64-bit word, bit i set for s_i = +1: reads,
// flips and the null test of an exchange are scalar operations.
struct SpinBits {
    uint64_t m;
    __device__ __forceinline__ void load(const int8_t* row, int N, int lane) {
        m = __ballot(lane < N && row[lane] > 0);
    }
    __device__ __forceinline__ int get(int i) const { return ((m >> i) & 1ull) ? 1 : -1; }
    __device__ __forceinline__ void flip(int i, int) { m ^= 1ull << i; }
    // spin at site 64 q + lane (0 past N)
    __device__ __forceinline__ int at(int q, int lane, int N) const {
        return (q == 0 && lane < N) ? (((m >> lane) & 1ull) ? 1 : -1) : 0;
    }
};
// The same interface over one site per lane and slot (N <= 256).
struct SpinLanes {
    WaveSpins w;
    __device__ __forceinline__ void load(const int8_t* row, int N, int lane) { w.load(row, N, lane); }
    __device__ __forceinline__ int get(int i) const { return w.get(i); }
    __device__ __forceinline__ void flip(int i, int lane) { w.set(i, -w.get(i), lane); }
    __device__ __forceinline__ int at(int q, int, int) const { return w.s[q]; }
};

// Rows of one whole [N][M] complex64 matrix through a single buffer descriptor: a row is a 32-bit scalar
// offset and the lanes' columns loop-invariant vector offsets (clamped to the row), so a proposal's loads
// need no 64-bit address arithmetic (the sweep here is bound by scalar issue, not by its row gathers).
struct MatRows {
    __amdgpu_buffer_rsrc_t r;
    int row_bytes;
};

__device__ __forceinline__ MatRows mat_rows(const float2* W, int N, int M) {
    return {__builtin_amdgcn_make_buffer_rsrc(const_cast<float2*>(W), (short)0, N * M * (int)sizeof(float2),
                                              0x00020000),
            M * (int)sizeof(float2)};
}

template <int E, bool PAIR>
__device__ __forceinline__ void mat_fetch(const MatRows& m, const unsigned (&loff)[E], int i, int j, float2 (&wi)[E],
                                          float2 (&wj)[E]) {
    const int oi = i * m.row_bytes, oj = j * m.row_bytes;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        wi[e] = __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(m.r, loff[e], oi, 0));
        if (PAIR) wj[e] = __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(m.r, loff[e], oj, 0));
    }
}

// Per-chain state of one wave.  theta of t~ changes only on accepted moves;
// its rows are fetched when a move is accepted and added at the next accepted
// move or measurement, so their L2 round trip overlaps the following proposals.
template <int E, bool PAIR, bool ONE>
struct BatchedChain {
    std::conditional_t<ONE, SpinBits, SpinLanes> sp;
    float ag[4];            // Re a of psi_gs at sites 64 q + lane
    float2 thg[E], tht[E];  // theta of psi_gs and of t~
    float Lg[E];            // Re log 2cosh theta_gs
    float2 pti[E], ptj[E];  // rows of t~'s W for the pending update of tht
    float pm;               // -2 s_i of the pending update, 0 when none
    float lu;               // ln(u) / 2 of this lane's draw: the acceptance test in the log domain
    float thp, thm;         // ONE: lu less the move's change of Re(a . s) of psi_gs, for s_i = +1 and -1
    int acc;                // lane l: accept bit of proposal 64 k + l of the current 64
    double m0, mr, mi;      // sums of |f|^2 and conj(f) beta r
};

// ln(u) / 2 from the hardware base-2 logarithm.  A move is accepted when u < |psi(s')/psi(s)|^2, that
// is when the change of Re log psi exceeds ln(u) / 2: the test compares that change with this
// threshold less the change of Re(a . s), so no exponential is taken per move (u = 0 gives -inf: accept).
__device__ __forceinline__ float half_ln(float u) {
    constexpr float kHalfLn2 = 0.34657359027997264f;  // ln(u)/2 = (ln 2 / 2) log2 u
    return kHalfLn2 * __builtin_amdgcn_logf(u);
}

// log 2cosh(zt) - log 2cosh(zg) of one unit (modulo 2 pi i): with s = sign Re z and w = exp(-2 s z),
// log 2cosh z = s z + log(1 + w), so the difference is st zt - sg zg + log((1 + wt) / (1 + wg)), one
// atan2 per unit.  |w| <= 1 comes from the hardware base-2 exponential (an error relative to |w|, so
// absolute and below 2^-21 in 1 + w), and the modulus part from two hardware base-2 logarithms of
// |1 + w|^2, which lies in [0, 4] (a zero of cosh gives -inf, as the library log of the quotient did).
__device__ __forceinline__ float2 unit_log_ratio(float2 zt, float2 zg) {
    constexpr float kM2Log2e = -2.8853900817779268f;  // exp(-2a) = 2^(-2a log2 e)
    constexpr float kHalfLn2 = 0.34657359027997264f;  // log(q)/2 = (ln 2 / 2) log2 q
    const float st = zt.x >= 0.f ? 1.f : -1.f, sg = zg.x >= 0.f ? 1.f : -1.f;
    const float et = __builtin_amdgcn_exp2f(fabsf(zt.x) * kM2Log2e), eg = __builtin_amdgcn_exp2f(fabsf(zg.x) * kM2Log2e);
    const float2 ct = cos_sin(2.f * st * zt.y), cg = cos_sin(2.f * sg * zg.y);
    const float2 a = make_float2(1.f + et * ct.x, -et * ct.y), b = make_float2(1.f + eg * cg.x, -eg * cg.y);
    const float2 q = make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);   // a conj(b)
    const float na = a.x * a.x + a.y * a.y, nb = b.x * b.x + b.y * b.y;
    const float lr = kHalfLn2 * (__builtin_amdgcn_logf(na) - __builtin_amdgcn_logf(nb));
    return make_float2(fabsf(zt.x) - fabsf(zg.x) + lr, st * zt.y - sg * zg.y + atan2f(q.y, q.x));
}

template <int E, bool PAIR, bool ONE>
__device__ __forceinline__ void apply_pending(BatchedChain<E, PAIR, ONE>& c, int lane, int M) {
    if (c.pm != 0.f) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const float2 d = row_delta<E, PAIR>(c.pti, c.ptj, e, lane, M);
            c.tht[e].x = fmaf(c.pm, d.x, c.tht[e].x);
            c.tht[e].y = fmaf(c.pm, d.y, c.tht[e].y);
        }
        c.pm = 0.f;
    }
}

// f_q(s) and the ratio t~(s)/psi_gs(s), added to the chain's sums.  Every sum runs in one fixed
// order that does not depend on how many lanes a chain has (the canonical order, shared with the
// grouped kernel below): per lane the slots in sequence (units 64 e + lane, sites 64 q + lane),
// then the lanes by bits 0 .. 5.  The unit terms are log 2cosh(theta_t) - log 2cosh(theta_gs) per
// unit (unit_log_ratio), the site terms (a_t - a_gs) s and e^{-i q.r} s / 2.
// ph: e^{-i q.r} and da: a_t - a_gs at this lane's sites
template <int E, bool PAIR, bool ONE>
__device__ __forceinline__ void measure(const BatchedArgs& A, BatchedChain<E, PAIR, ONE>& c, const float2 (&ph)[4],
                                        const float2 (&da)[4], double2 beta, int lane) {
    const int N = A.N, M = A.M;
    apply_pending(c, lane, M);
    float2 f = make_float2(0.f, 0.f), dA = make_float2(0.f, 0.f), dU = make_float2(0.f, 0.f);
#pragma unroll
    for (int qq = 0; qq < 4; ++qq) {
        const int site = qq * kWave + lane;
        if (site < N) {
            const float s = (float)c.sp.at(qq, lane, N);
            f = cadd(f, cscale(ph[qq], 0.5f * s));
            dA = cadd(dA, cscale(da[qq], s));
        }
    }
#pragma unroll
    for (int e = 0; e < E; ++e)
        if (e * kWave + lane < M) dU = cadd(dU, unit_log_ratio(c.tht[e], c.thg[e]));
    f = make_float2(wave_total(f.x), wave_total(f.y));
    const float2 dlog = make_float2(wave_total(dU.x) + wave_total(dA.x), wave_total(dU.y) + wave_total(dA.y));
    const float2 r = cscale(cos_sin(dlog.y), expf(dlog.x));
    const double fx = (double)f.x * (1.0 / sqrt((double)N)), fy = (double)f.y * (1.0 / sqrt((double)N));
    const double2 br = zmul(beta, make_double2((double)r.x, (double)r.y));
    c.m0 += fx * fx + fy * fy;
    c.mr += fx * br.x + fy * br.y;  // conj(f) * (beta r)
    c.mi += fx * br.y - fy * br.x;
}

// Trace words of the `count` proposals t0 .. t0 + count - 1 (t0 a multiple of 64) from their accept
// bits, one per lane.
template <int E, bool PAIR, bool ONE>
__device__ __forceinline__ void flush_accepts(BatchedChain<E, PAIR, ONE>& c, uint32_t* trow, int t0, int count,
                                              int lane) {
    if (trow) {
        const uint64_t bits = __ballot(c.acc != 0);
        if (lane == 0) {
            trow[t0 >> 5] = (uint32_t)bits;
            if (count > 32) trow[(t0 >> 5) + 1] = (uint32_t)(bits >> 32);
        }
    }
    c.acc = 0;
}

// Proposal t of chain g.  Rows of psi_gs are read only for live moves; with LDSG from LDS (s_w: rows
// of E 64 columns that hold zeros past M).  Every 64th proposal draws the next 64 (one per lane) with
// their thresholds ln(u)/2 (with ONE less each draw's change of Re(a . s), for both signs of s_i), and
// writes the accept bits of the previous 64 to the trace.  The move is accepted when the wave total of
// the log-cosh change exceeds ln(u)/2 less the change of Re(a . s), the same test in every kernel here.
template <int E, bool PAIR, bool ONE, bool LDSG>
__device__ __forceinline__ void batched_step(const BatchedArgs& A, const float2* s_w, uint64_t g, int lane, int t,
                                             BatchedChain<E, PAIR, ONE>& c, const MatRows& Wg, const MatRows& Wt,
                                             const unsigned (&loff)[E], uint32_t* trow, DrawBatch& batch) {
    const int N = A.N, M = A.M;
    const int l = t & 63;
    if (l == 0) {
        if (t > 0) flush_accepts(c, trow, t - 64, 64, lane);
        batch = draw_batch(A.seed, (uint32_t)g, (uint64_t)t, lane, N);
        c.lu = half_ln(batch.u);
        if (ONE) {
            // Re a of psi_gs at this lane's sites i, j (site k sits in lane k): the move changes
            // Re(a . s) by -2 s_i (a_i - a_j), or by -2 s_i a_i for a flip, that is by -s_i d2 (exactly
            // as -2 s_i a_i + 2 s_i a_j rounds)
            const float ai = __int_as_float(__builtin_amdgcn_ds_bpermute(batch.i << 2, __float_as_int(c.ag[0])));
            const float aj = __int_as_float(__builtin_amdgcn_ds_bpermute(batch.j << 2, __float_as_int(c.ag[0])));
            const float d2 = PAIR ? 2.f * (ai - aj) : 2.f * ai;
            c.thp = c.lu + d2;   // s_i = +1: the change is -d2
            c.thm = c.lu - d2;
        }
    }
    Proposal cur = proposal_at(batch, l);
    const int si = c.sp.get(cur.i), sj = c.sp.get(cur.j);
    if (!(PAIR && si == sj)) {
        float2 wi[E], wj[E], tn[E];
        float Ln[E];
        float total, thr;
        if (LDSG) {
            constexpr int Mp = E * kWave;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                wi[e] = s_w[cur.i * Mp + e * kWave + lane];
                if (PAIR) wj[e] = s_w[cur.j * Mp + e * kWave + lane];
            }
        } else {
            mat_fetch<E, PAIR>(Wg, loff, cur.i, cur.j, wi, wj);
        }
        if (ONE) {
            total = units_dlog<E, PAIR, !LDSG>(si, wi, wj, c.thg, c.Lg, tn, Ln, lane, M);
            thr = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(si > 0 ? c.thp : c.thm), l));
        } else {
            const float m2si = -2.f * (float)si;
            float da = m2si * site_value<ONE>(c.ag, cur.i);
            if (PAIR) da -= m2si * site_value<ONE>(c.ag, cur.j);
            total = units_dlog<E, PAIR>(si, wi, wj, c.thg, c.Lg, tn, Ln, lane, M);
            thr = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(c.lu), l)) - uniform(da);
        }
        if (total > thr) {
#pragma unroll
            for (int e = 0; e < E; ++e) { c.thg[e] = tn[e]; c.Lg[e] = Ln[e]; }
            apply_pending(c, lane, M);
            mat_fetch<E, PAIR>(Wt, loff, cur.i, cur.j, c.pti, c.ptj);
            c.pm = -2.f * (float)si;
            c.sp.flip(cur.i, lane);
            if (PAIR) c.sp.flip(cur.j, lane);
            if (trow) c.acc = lane == l ? 1 : c.acc;
        }
    }
}
// Four waves per SIMD (at most 128 registers) for the small chain widths, which hides more of each
// wave's dependency stalls.  LDSG: the block first copies W of psi_gs ([N][M] complex64, rows padded
// with zeros to E 64 columns) into LDS after its spin rows, and live proposals read their rows there.
template <int E, bool PAIR, bool ONE, bool LDSG>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(E <= 2 ? 4 : 1)))
void k_batched(BatchedArgs A) {
    extern __shared__ int8_t s_spins[];           // one 256-byte row per wave, then W of psi_gs (LDSG)
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    int8_t* row = s_spins + wv * 256;
    const int N = A.N, M = A.M;
    float2* s_w = reinterpret_cast<float2*>(s_spins + 256 * (blockDim.x >> 6));
    if (LDSG) {
        constexpr int Mp = E * kWave;   // rows padded to the lanes' units, zeros past M
        for (int k = threadIdx.x; k < N * Mp; k += blockDim.x) {
            const int i = k / Mp, col = k % Mp;
            s_w[k] = col < M ? A.gs.W[(long)i * M + col] : make_float2(0.f, 0.f);
        }
        __syncthreads();
    }
    const long wave_id = (long)blockIdx.x * (blockDim.x >> 6) + wv;
    const unsigned long long t_start = A.clocks ? wall_clock64() : 0ull;
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
        BatchedChain<E, PAIR, ONE> c;
        c.sp.load(row, N, lane);
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) {
            const int site = qq * kWave + lane;
            c.ag[qq] = site < N ? A.gs.a[site].x : 0.f;
        }

        // theta of psi_gs and of t~_inst from the spins (lanes past M: theta = 0, see proposal_dlog)
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int k = e * kWave + lane;
            c.thg[e] = (k < M) ? A.gs.b[k] : make_float2(0.f, 0.f);
            c.tht[e] = (k < M) ? bt[k] : make_float2(0.f, 0.f);
        }
#pragma unroll 2
        for (int i = 0; i < N; ++i) {
            const float si = (float)c.sp.get(i);
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int k = e * kWave + lane;
                const long at_ik = (long)i * M + min(k, M - 1);
                const float2 wg = A.gs.W[at_ik], wt = Wt[at_ik];
                const float s = (k < M) ? si : 0.f;
                c.thg[e].x = fmaf(s, wg.x, c.thg[e].x);
                c.thg[e].y = fmaf(s, wg.y, c.thg[e].y);
                c.tht[e].x = fmaf(s, wt.x, c.tht[e].x);
                c.tht[e].y = fmaf(s, wt.y, c.tht[e].y);
            }
        }
#pragma unroll
        for (int e = 0; e < E; ++e) c.Lg[e] = re_log2cosh_fast(c.thg[e]);
        // phases e^{-i q.r} of this lane's sites (q.r reduced to [-pi, pi] in double, then cos_sin of
        // the float, accurate there) and a_t - a_gs there
        float2 ph[4], da[4];
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) {
            const int site = qq * kWave + lane;
            ph[qq] = make_float2(0.f, 0.f);
            da[qq] = make_float2(0.f, 0.f);
            if (site < N) {
                da[qq] = csub(at[site], A.gs.a[site]);
                const int x = A.kind == 0 ? site : site % A.Lx;
                const int y = A.kind == 0 ? 0 : site / A.Lx;
                const double arg = q0 * x + q1 * y;
                const double two_pi = 6.283185307179586476925286766559;
                const float red = (float)(arg - two_pi * rint(arg / two_pi));
                const float2 cs = cos_sin(red);
                ph[qq] = make_float2(cs.x, -cs.y);
            }
        }
        const double2 beta = A.betas[inst];
        c.pm = 0.f;
        c.lu = c.thp = c.thm = 0.f;
        c.acc = 0;
        c.m0 = c.mr = c.mi = 0.0;
        uint32_t* trow = A.trace ? A.trace + (long)g * A.trace_words : nullptr;
        const int total = (A.n_burn + A.n_sweeps) * N;   // the plan checks that it fits
        const MatRows Wg = mat_rows(A.gs.W, N, M), Wtr = mat_rows(Wt, N, M);
        unsigned loff[E];
#pragma unroll
        for (int e = 0; e < E; ++e) loff[e] = (unsigned)min(e * kWave + lane, M - 1) * (unsigned)sizeof(float2);
        DrawBatch batch;
        int t = 0;
        for (int sw = 0; sw < A.n_burn + A.n_sweeps; ++sw) {
            for (int p = 0; p < N; ++p, ++t) batched_step<E, PAIR, ONE, LDSG>(A, s_w, g, lane, t, c, Wg, Wtr, loff, trow, batch);
            if (sw >= A.n_burn) measure(A, c, ph, da, beta, lane);
        }
        if (total > 0) flush_accepts(c, trow, (total - 1) & ~63, total - ((total - 1) & ~63), lane);
        if (lane == 0) {
            A.partial[2 * g] = make_double2(c.m0, 0.0);
            A.partial[2 * g + 1] = make_double2(c.mr, c.mi);
        }
    }
    // profiling: when this wave started and when it found no chain left (the tail of the launch)
    if (A.clocks && lane == 0 && wave_id < CRBM_MAX_CLOCK_WAVES) {
        A.clocks[2 * wave_id] = t_start;
        A.clocks[2 * wave_id + 1] = wall_clock64();
    }
}

// ------------------------------------------------------------------ several chains per wave
// A chain on L = 16 or 32 lanes (G = 64 / L chains per wave, one per lane group), for M <= 128 (L = 16)
// or 256 (L = 32): every lane holds EL = E64 64 / L units, so the per-proposal control (draw, site
// values, reduction, accept) is shared by G proposals of G chains.  Lane gl of a group holds the
// units and sites 64 e + L j + gl, j < 64 / L: sums run over the slots e in sequence for each j, then
// over the lane bits 0 .. log2 L - 1 (DPP within the row, a swap across rows for L = 32), then over
// j by its bits, which is the 64-lane kernel's order exactly, so both give the same decisions and
// moments bit for bit.  The group's spins live in LDS (row per chain); the group's first lane writes
// them.  Groups step in lockstep; a group without a chain (the grid's last round) runs masked.

// sum over the L lanes of each group by lane bits 0 .. log2 L - 1; every lane of the group ends with
// the same value.  All 64 lanes must be active.
template <int L>
__device__ __forceinline__ float group_sum(float v) {
    v += dpp_move<0xB1, 0xF>(v);   // bit 0: quad_perm [1, 0, 3, 2]
    v += dpp_move<0x4E, 0xF>(v);   // bit 1: quad_perm [2, 3, 0, 1]
    v += dpp_move<0x141, 0xF>(v);  // bit 2: row_half_mirror
    v += dpp_move<0x140, 0xF>(v);  // bit 3: row_mirror
    if (L == 32) v += __shfl_xor(v, 16, kWave);   // bit 4
    return v;
}
// canonical total of per-lane partials over sub-slots j (lane bits log2 L .. 5)
template <int L>
__device__ __forceinline__ float group_total(const float (&p)[64 / L]) {
    if (L == 32) return group_sum<L>(p[0]) + group_sum<L>(p[1]);
    const float a = group_sum<L>(p[0]) + group_sum<L>(p[1]);
    const float b = group_sum<L>(p[2]) + group_sum<L>(p[3]);
    return a + b;
}

// e^{-i q.r} at a site (q.r reduced to [-pi, pi] in double, then cos_sin of the float)
__device__ __forceinline__ float2 site_phase(const BatchedArgs& A, int site, double q0, double q1) {
    const int x = A.kind == 0 ? site : site % A.Lx;
    const int y = A.kind == 0 ? 0 : site / A.Lx;
    const double arg = q0 * x + q1 * y;
    const double two_pi = 6.283185307179586476925286766559;
    const float red = (float)(arg - two_pi * rint(arg / two_pi));
    const float2 cs = cos_sin(red);
    return make_float2(cs.x, -cs.y);
}

template <int L, int E64, bool PAIR>
__global__ __launch_bounds__(512) void k_batched_grp(BatchedArgs A) {
    constexpr int G = kWave / L;        // chains per wave
    constexpr int J = kWave / L;        // sub-slots per lane
    constexpr int EL = E64 * J;         // units per lane, slot k = e J + j: unit 64 e + L j + gl
    extern __shared__ int8_t s_spins[];  // one 256-byte row per chain
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int grp = lane / L, gl = lane % L;
    int8_t* row = s_spins + (wv * G + grp) * 256;
    const int N = A.N, M = A.M;
    const long wave_id = (long)blockIdx.x * (blockDim.x >> 6) + wv;
    const unsigned long long t_start = A.clocks ? wall_clock64() : 0ull;
    const float* gsa = reinterpret_cast<const float*>(A.gs.a);
    for (;;) {
        unsigned long long g0 = 0;
        if (lane == 0) g0 = atomicAdd(A.counter, (unsigned long long)G);
        g0 = (unsigned long long)__builtin_amdgcn_readfirstlane((int)(g0 & 0xFFFFFFFFull)) |
             ((unsigned long long)__builtin_amdgcn_readfirstlane((int)(g0 >> 32)) << 32);
        if ((int64_t)g0 >= A.total) break;
        const int64_t g = (int64_t)g0 + grp;
        const bool act = g < A.total;
        const int64_t gq = act ? g : A.total - 1;
        int lo = 0, hi = A.n_inst;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (A.offsets[mid] <= gq) lo = mid; else hi = mid;
        }
        const int inst = lo;
        const float2* tp = A.t_params + (long)inst * A.P;
        const float2* at = tp;
        const float2* bt = tp + N;
        const float2* Wt = tp + N + M;
        const double q0 = A.q[2 * inst], q1 = A.q[2 * inst + 1];

        // Fisher-Yates start at total S^z = 0 (Philox tag 1, counter a = chain id), by the group's first lane
        if (gl == 0) {
            for (int i = 0; i < N; ++i) row[i] = (i < N / 2) ? 1 : -1;
            if (act)
                for (int k = N - 1; k >= 1; --k) {
                    const int m = draw_index(draw(A.seed, (uint32_t)g, (uint64_t)k, 1u).x, k + 1);
                    const int8_t t = row[k];
                    row[k] = row[m];
                    row[m] = t;
                }
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

        float2 thg[EL], tht[EL];
        float Lg[EL];
        // slot k holds unit u = 64 (k / J) + L (k % J) + gl; its column clamped to the row is col(k)
        auto col = [&](int k) { return min(kWave * (k / J) + L * (k % J) + gl, M - 1); };
#pragma unroll
        for (int k = 0; k < EL; ++k) {
            const int u = kWave * (k / J) + L * (k % J) + gl;
            thg[k] = (u < M) ? A.gs.b[u] : make_float2(0.f, 0.f);
            tht[k] = (u < M) ? bt[u] : make_float2(0.f, 0.f);
        }
#pragma unroll 1
        for (int i = 0; i < N; ++i) {
            const float si = (float)row[i];
#pragma unroll
            for (int k = 0; k < EL; ++k) {
                const int u = kWave * (k / J) + L * (k % J) + gl;
                const float2 wg = A.gs.W[(long)i * M + col(k)], wt = Wt[(long)i * M + col(k)];
                const float sv = (u < M) ? si : 0.f;
                thg[k].x = fmaf(sv, wg.x, thg[k].x);
                thg[k].y = fmaf(sv, wg.y, thg[k].y);
                tht[k].x = fmaf(sv, wt.x, tht[k].x);
                tht[k].y = fmaf(sv, wt.y, tht[k].y);
            }
        }
#pragma unroll
        for (int k = 0; k < EL; ++k) Lg[k] = re_log2cosh_fast(thg[k]);
        const double2 beta = A.betas[inst];
        float2 pt[EL];      // pending change of theta_t per unit of pm: W_t rows i (- j) of the last accepted move
        float pm = 0.f;
        uint32_t tw = 0;
        double m0 = 0.0, mr = 0.0, mi = 0.0;
        uint32_t* trow = (A.trace && act) ? A.trace + (long)g * A.trace_words : nullptr;
        const int total = (A.n_burn + A.n_sweeps) * N;
        int bi = 0, bj = 0;
        float bu = 0.f;
        auto apply = [&]() {
            if (pm != 0.f) {
#pragma unroll
                for (int k = 0; k < EL; ++k) {
                    tht[k].x = fmaf(pm, pt[k].x, tht[k].x);
                    tht[k].y = fmaf(pm, pt[k].y, tht[k].y);
                }
                pm = 0.f;
            }
        };
        int t = 0;
        for (int sw = 0; sw < A.n_burn + A.n_sweeps; ++sw) {
            for (int p = 0; p < N; ++p, ++t) {
                // proposal t: the group's lane t % L drew it (counter t of the chain's stream, tag 0)
                if ((t % L) == 0) {
                    uint32_t k0 = (uint32_t)A.seed, k1 = (uint32_t)(A.seed >> 32);
                    asm volatile("" : "+s"(k0), "+s"(k1));
                    const uint64_t tt = (uint64_t)(t + gl);
                    const u32x4 x = philox4x32_10((uint32_t)gq, (uint32_t)tt, (uint32_t)(tt >> 32), 0u, k0, k1);
                    bi = draw_index(x.x, N);
                    bj = draw_index(x.y, N);
                    bu = draw_unit(x.z);
                }
                const int src = grp * L + (t % L);
                const int ci = __shfl(bi, src, kWave), cj = __shfl(bj, src, kWave);
                const float cu = __shfl(bu, src, kWave);
                const int si = row[ci], sj = row[cj];
                const bool live = act && !(PAIR && si == sj);
                bool acc = false;
                if (__builtin_amdgcn_ballot_w64(live)) {
                    float2 wi[EL], wj[EL], tn[EL];
                    float Ln[EL];
                    const float ai = gsa[2 * ci];
                    const float aj = PAIR ? gsa[2 * cj] : 0.f;
#pragma unroll
                    for (int k = 0; k < EL; ++k) {
                        wi[k] = A.gs.W[(long)ci * M + col(k)];
                        if (PAIR) wj[k] = A.gs.W[(long)cj * M + col(k)];
                    }
                    const float m2si = -2.f * (float)si;
                    float ds[J];
#pragma unroll
                    for (int j = 0; j < J; ++j) ds[j] = 0.f;
#pragma unroll
                    for (int k = 0; k < EL; ++k) {
                        const int u = kWave * (k / J) + L * (k % J) + gl;
                        float2 d = PAIR ? csub(wi[k], wj[k]) : wi[k];
                        if (u >= M) d = make_float2(0.f, 0.f);
                        tn[k].x = fmaf(m2si, d.x, thg[k].x);
                        tn[k].y = fmaf(m2si, d.y, thg[k].y);
                        Ln[k] = re_log2cosh_fast(tn[k]);
                        ds[k % J] += Ln[k] - Lg[k];
                    }
                    float da = m2si * ai;
                    if (PAIR) da -= m2si * aj;
                    acc = live && (group_total<L>(ds) > half_ln(cu) - da);
                    if (acc) {
#pragma unroll
                        for (int k = 0; k < EL; ++k) { thg[k] = tn[k]; Lg[k] = Ln[k]; }
                        apply();
#pragma unroll
                        for (int k = 0; k < EL; ++k) {
                            const int u = kWave * (k / J) + L * (k % J) + gl;
                            const float2 ri = Wt[(long)ci * M + col(k)];
                            float2 d = ri;
                            if (PAIR) d = csub(ri, Wt[(long)cj * M + col(k)]);
                            pt[k] = (u < M) ? d : make_float2(0.f, 0.f);
                        }
                        pm = m2si;
                        if (gl == 0) {
                            row[ci] = (int8_t)(-si);
                            if (PAIR) row[cj] = (int8_t)(-sj);
                        }
                    }
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
                }
                if (acc) tw |= 1u << (t & 31);
                if ((t & 31) == 31) {
                    if (trow && gl == 0) trow[t >> 5] = tw;
                    tw = 0;
                }
            }
            if (sw >= A.n_burn) {
                // the measurement in the canonical order (see measure above): per sub-slot j the slots in
                // sequence, the group's lanes, then the sub-slots by their bits
                apply();
                float fx_[J], fy_[J], ax_[J], ay_[J], ux_[J], uy_[J];
#pragma unroll
                for (int j = 0; j < J; ++j) {
                    float fx = 0.f, fy = 0.f, ax = 0.f, ay = 0.f, ux = 0.f, uy = 0.f;
#pragma unroll 1
                    for (int qq = 0; qq < 4; ++qq) {
                        const int site = kWave * qq + L * j + gl;
                        if (site < N) {
                            const float sv = (float)row[site];
                            const float2 ph = site_phase(A, site, q0, q1);
                            const float2 da = csub(at[site], A.gs.a[site]);
                            const float2 fc = cscale(ph, 0.5f * sv), dc = cscale(da, sv);
                            fx += fc.x; fy += fc.y;
                            ax += dc.x; ay += dc.y;
                        }
                    }
#pragma unroll
                    for (int e = 0; e < E64; ++e) {
                        const int k = e * J + j;
                        if (kWave * e + L * j + gl < M) {
                            const float2 d = unit_log_ratio(tht[k], thg[k]);
                            ux += d.x;
                            uy += d.y;
                        }
                    }
                    fx_[j] = fx; fy_[j] = fy; ax_[j] = ax; ay_[j] = ay; ux_[j] = ux; uy_[j] = uy;
                }
                const float2 f = make_float2(group_total<L>(fx_), group_total<L>(fy_));
                const float2 dlog = make_float2(group_total<L>(ux_) + group_total<L>(ax_),
                                                group_total<L>(uy_) + group_total<L>(ay_));
                const float2 r = cscale(cos_sin(dlog.y), expf(dlog.x));
                const double fx = (double)f.x * (1.0 / sqrt((double)N)), fy = (double)f.y * (1.0 / sqrt((double)N));
                const double2 br = zmul(beta, make_double2((double)r.x, (double)r.y));
                m0 += fx * fx + fy * fy;
                mr += fx * br.x + fy * br.y;
                mi += fx * br.y - fy * br.x;
            }
        }
        if (act && gl == 0) {
            A.partial[2 * g] = make_double2(m0, 0.0);
            A.partial[2 * g + 1] = make_double2(mr, mi);
            if (trow && (total & 31) != 0) trow[total >> 5] = tw;
        }
        __builtin_amdgcn_wave_barrier();
    }
    if (A.clocks && lane == 0 && wave_id < CRBM_MAX_CLOCK_WAVES) {
        A.clocks[2 * wave_id] = t_start;
        A.clocks[2 * wave_id + 1] = wall_clock64();
    }
}

// mu_out[i] = (sum of chain partials of instance i) / (c_i n_sweeps).  An instance whose chain range
// [offsets[i], offsets[i+1]) is not inside [0, total) reads no partials and gets NaN moments.
__global__ void k_batched_reduce(const double2* __restrict__ partial, const int64_t* __restrict__ offsets, int n_inst,
                                 int64_t total, int n_sweeps, double2* __restrict__ mu) {
    const int i = blockIdx.x;
    if (i >= n_inst) return;
    __shared__ double sh[4][4];
    const int64_t b = offsets[i], e = offsets[i + 1];
    if (b < 0 || e < b || e > total) {
        if (threadIdx.x == 0) {
            const double nan = __builtin_nan("");
            mu[2 * i] = make_double2(nan, nan);
            mu[2 * i + 1] = make_double2(nan, nan);
        }
        return;
    }
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

bool batched_lanes_ok(int lanes, int M) {
    if (lanes == kWave) return true;
    const int E64 = (M + kWave - 1) / kWave;
    return (lanes == 32 && E64 <= 4) || (lanes == 16 && E64 <= 2);
}

// Blocks of k that one compute unit holds with `lds` bytes of dynamic LDS (0 when the query fails).
template <typename K>
static int resident_blocks(K k, int threads, size_t lds) {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, threads, lds) != hipSuccess) return 0;
    return n;
}

// Whether k_batched<E, PAIR, ONE> keeps its copy of psi_gs's W in LDS: W fits (E <= 4, N E 64
// complex64 with the spin rows at most the compute unit's LDS) and the compute unit then holds as
// many blocks as without it.
template <int E, bool PAIR, bool ONE>
static bool lds_rows_for(int N, int M, int waves_per_block) {
    if constexpr (E > 4) {
        return false;
    } else {
        const size_t lds = 256 * (size_t)waves_per_block, lds_w = lds + (size_t)N * E * kWave * sizeof(float2);
        if (lds_w > (size_t)kMaxBatchedLds) return false;
        // raise the kernel's dynamic LDS limit once per device (the first call on each)
        static signed char attr[kMaxDevices] = {};
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return false;
        if (attr[dev] == 0)
            attr[dev] = hipFuncSetAttribute((const void*)k_batched<E, PAIR, ONE, true>,
                                            hipFuncAttributeMaxDynamicSharedMemorySize, kMaxBatchedLds) == hipSuccess
                            ? 1 : -1;
        if (attr[dev] < 0) return false;
        const int threads = kWave * waves_per_block;
        const int with = resident_blocks(k_batched<E, PAIR, ONE, true>, threads, lds_w);
        return with > 0 && with >= resident_blocks(k_batched<E, PAIR, ONE, false>, threads, lds);
    }
}

template <int E, bool PAIR, bool ONE>
static void launch_one_batched(const BatchedArgs& A, int blocks, int waves_per_block, hipStream_t stream) {
    const dim3 grid(blocks), block(kWave * waves_per_block);
    const size_t lds = 256 * (size_t)waves_per_block;
    if (lds_rows_for<E, PAIR, ONE>(A.N, A.M, waves_per_block))
        hipLaunchKernelGGL((k_batched<E, PAIR, ONE, true>), grid, block,
                           lds + (size_t)A.N * E * kWave * sizeof(float2), stream, A);
    else
        hipLaunchKernelGGL((k_batched<E, PAIR, ONE, false>), grid, block, lds, stream, A);
}

bool batched_lds_rows(int N, int M, int proposal, int waves_per_block) {
    const int E = (M + kWave - 1) / kWave;
    const bool pair = proposal == 1, one = N <= kWave;
    switch (E) {
#define CRBM_CASE(e)                                                           \
    case e:                                                                    \
        if (pair && one) return lds_rows_for<e, true, true>(N, M, waves_per_block);   \
        if (pair) return lds_rows_for<e, true, false>(N, M, waves_per_block);         \
        if (one) return lds_rows_for<e, false, true>(N, M, waves_per_block);          \
        return lds_rows_for<e, false, false>(N, M, waves_per_block);
        CRBM_CASE(1) CRBM_CASE(2) CRBM_CASE(3) CRBM_CASE(4)
#undef CRBM_CASE
        default: return false;
    }
}

hipError_t launch_batched(const BatchedArgs& A, int blocks, int waves_per_block, int lanes, double2* mu,
                          hipStream_t stream) {
    if (!batched_lanes_ok(lanes, A.M)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_batched_reset, dim3(1), dim3(64), 0, stream, A.counter);
    const int E = (A.M + kWave - 1) / kWave;
    const dim3 grid(blocks), block(64 * waves_per_block);
    const bool pair = A.proposal == 1, one = A.N <= kWave;
    if (lanes != kWave) {
        const size_t lds_g = 256 * (size_t)waves_per_block * (kWave / lanes);
#define CRBM_GRP(l, e)                                                                                    \
    if (lanes == l && E == e) {                                                                           \
        if (pair) hipLaunchKernelGGL((k_batched_grp<l, e, true>), grid, block, lds_g, stream, A);         \
        else hipLaunchKernelGGL((k_batched_grp<l, e, false>), grid, block, lds_g, stream, A);             \
    }
        CRBM_GRP(16, 1) CRBM_GRP(16, 2) CRBM_GRP(32, 1) CRBM_GRP(32, 2) CRBM_GRP(32, 3) CRBM_GRP(32, 4)
#undef CRBM_GRP
        hipLaunchKernelGGL(k_batched_reduce, dim3(A.n_inst), dim3(256), 0, stream, A.partial, A.offsets, A.n_inst,
                           (int64_t)A.total, A.n_sweeps, mu);
        return hipGetLastError();
    }
    switch (E) {
#define CRBM_CASE(e)                                                                              \
    case e:                                                                                       \
        if (pair && one) launch_one_batched<e, true, true>(A, blocks, waves_per_block, stream);   \
        else if (pair) launch_one_batched<e, true, false>(A, blocks, waves_per_block, stream);    \
        else if (one) launch_one_batched<e, false, true>(A, blocks, waves_per_block, stream);     \
        else launch_one_batched<e, false, false>(A, blocks, waves_per_block, stream);             \
        break;
        CRBM_CASE(1) CRBM_CASE(2) CRBM_CASE(3) CRBM_CASE(4) CRBM_CASE(5) CRBM_CASE(6) CRBM_CASE(7) CRBM_CASE(8)
#undef CRBM_CASE
        default: return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL(k_batched_reduce, dim3(A.n_inst), dim3(256), 0, stream, A.partial, A.offsets, A.n_inst,
                       (int64_t)A.total, A.n_sweeps, mu);
    return hipGetLastError();
}

}  // namespace crbm
