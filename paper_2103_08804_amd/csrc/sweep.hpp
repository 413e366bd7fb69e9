// Metropolis proposals shared by the sweep and the batched moments.
//
// A proposal flips site i (or, for an exchange, sites i and j with
// s_i = -s_j) and is accepted on u < |psi'/psi|^2 (Sec. III).  Sites and
// uniform come from the chain's counter-based stream alone, so 64 proposals
// are drawn at once, one per lane.  An exchange of equal spins is a null move
// and reads nothing; a live move reads rows W_i (and W_j) with every load
// issued before the first use.  Row reads use a clamped column: lanes past M
// read column M - 1 and the caller adds zero for them.  The sweep is bound by
// these row gathers (L2 hits), which is why null moves must not issue them.
#pragma once
#include "device.hpp"
#include "internal.hpp"

namespace crbm {

struct Proposal {
    int i, j;      // sites (wave-uniform)
    float u;       // acceptance uniform
    float ai, aj;  // Re a_i, Re a_j
};

// Draws of 64 consecutive proposals t0 + l, one per lane l (counter t0 + l of stream `chain`,
// Philox tag 0): the generator runs on the vector unit once per 64 proposals, and a proposal
// takes its sites and uniform from its lane with readlane.
struct DrawBatch {
    int i, j;
    float u;
};

__device__ __forceinline__ DrawBatch draw_batch(uint64_t seed, uint32_t chain, uint64_t t0, int lane, int N) {
    uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    // An empty statement that marks the key as rewritten here: the ten round keys are then derived at
    // each batch (20 scalar adds per 64 proposals) instead of being hoisted out of the sweep loop,
    // where they would hold 20 scalar registers for the whole launch and push others into spills.
    asm volatile("" : "+s"(k0), "+s"(k1));
    const uint64_t t = t0 + (uint64_t)lane;
    const u32x4 x = philox4x32_10(chain, (uint32_t)t, (uint32_t)(t >> 32), 0u, k0, k1);
    return {draw_index(x.x, N), draw_index(x.y, N), draw_unit(x.z)};
}

__device__ __forceinline__ Proposal proposal_at(const DrawBatch& b, int l) {
    return {__builtin_amdgcn_readlane(b.i, l), __builtin_amdgcn_readlane(b.j, l),
            __int_as_float(__builtin_amdgcn_readlane(__float_as_int(b.u), l)), 0.f, 0.f};
}

// proposal t (counted from t0 of the first batch) out of the batch, drawing the next batch at
// every 64th proposal
__device__ __forceinline__ Proposal next_proposal(DrawBatch& b, uint64_t seed, uint32_t chain, uint64_t t0, long t,
                                                  int lane, int N) {
    if ((t & 63) == 0) b = draw_batch(seed, chain, t0 + (uint64_t)t, lane, N);
    return proposal_at(b, (int)(t & 63));
}

// Raw buffer descriptor of one W row (M complex64): the row base stays in scalar registers and each
// load takes a loop-invariant 32-bit byte offset per lane.  Word 3 selects 32-bit untyped data.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const float2* row, int M) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<float2*>(row), (short)0, M * (int)sizeof(float2),
                                             0x00020000);
}

__device__ __forceinline__ float2 row_load(__amdgpu_buffer_rsrc_t r, unsigned off) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
    return __builtin_bit_cast(float2, v);
}

// byte offset of this lane's element k = 64 e + lane, clamped to the row (lanes past M re-read
// column M - 1; callers add zero for them)
__device__ __forceinline__ unsigned lane_offset(int e, int lane, int M) {
    return (unsigned)min(e * kWave + lane, M - 1) * (unsigned)sizeof(float2);
}

// lane's elements k = 64 e + lane of rows i (and j) of an [N][M] complex64 matrix
template <int E, bool PAIR>
__device__ __forceinline__ void fetch_w(const float2* __restrict__ W, int M, int i, int j, int lane, float2 (&wi)[E],
                                        float2 (&wj)[E]) {
    const __amdgpu_buffer_rsrc_t ri = row_rsrc(W + (long)i * M, M);
    const __amdgpu_buffer_rsrc_t rj = row_rsrc(W + (long)j * M, M);
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const unsigned off = lane_offset(e, lane, M);
        wi[e] = row_load(ri, off);
        if (PAIR) wj[e] = row_load(rj, off);
    }
}

template <int E, bool PAIR>
__device__ __forceinline__ void fetch_rows(const RbmView& psi, int M, Proposal& q, int lane, float2 (&wi)[E],
                                           float2 (&wj)[E]) {
    q.ai = psi.a[q.i].x;
    q.aj = PAIR ? psi.a[q.j].x : 0.f;
    fetch_w<E, PAIR>(psi.W, M, q.i, q.j, lane, wi, wj);
}

// change of theta_k per unit of -2 s_i: W_ik (flip) or W_ik - W_jk (exchange); zero past M.
// E = ceil(M / 64), so only the last group can hold lanes past M.  MASK = false for rows that hold
// zeros past M themselves.
template <int E, bool PAIR, bool MASK = true>
__device__ __forceinline__ float2 row_delta(const float2 (&wi)[E], const float2 (&wj)[E], int e, int lane, int M) {
    float2 d = PAIR ? csub(wi[e], wj[e]) : wi[e];
    if (MASK && e == E - 1 && e * kWave + lane >= M) d = make_float2(0.f, 0.f);
    return d;
}

// theta' = theta - 2 s_i d and the wave total of the change of Re log 2cosh theta.  Lanes past M
// hold theta = 0 and L = Re log 2cosh(0) from the same function, so they add exactly zero.
template <int E, bool PAIR, bool MASK = true>
__device__ __forceinline__ float units_dlog(int si, const float2 (&wi)[E], const float2 (&wj)[E],
                                            const float2 (&th)[E], const float (&L)[E], float2 (&tn)[E],
                                            float (&Ln)[E], int lane, int M) {
    const float m2si = -2.f * (float)si;
    float dsum = 0.f;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const float2 d = row_delta<E, PAIR, MASK>(wi, wj, e, lane, M);
        tn[e].x = fmaf(m2si, d.x, th[e].x);
        tn[e].y = fmaf(m2si, d.y, th[e].y);
        Ln[e] = re_log2cosh_fast(tn[e]);
        const float x = Ln[e] - L[e];
        dsum = e == 0 ? x : dsum + x;   // 0 + x would only change the sign of a zero
    }
    return wave_total(dsum);
}

// ... plus the change of Re(a . s): the change of Re log psi of the move (wave-uniform)
template <int E, bool PAIR>
__device__ __forceinline__ float proposal_dlog(const Proposal& q, int si, const float2 (&wi)[E],
                                               const float2 (&wj)[E], const float2 (&th)[E], const float (&L)[E],
                                               float2 (&tn)[E], float (&Ln)[E], int lane, int M) {
    const float m2si = -2.f * (float)si;
    float da = m2si * q.ai;
    if (PAIR) da -= m2si * q.aj;
    return units_dlog<E, PAIR>(si, wi, wj, th, L, tn, Ln, lane, M) + uniform(da);
}

}  // namespace crbm
