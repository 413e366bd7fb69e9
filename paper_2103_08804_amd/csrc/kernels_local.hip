// theta GEMM, per-sample local estimators and Chebyshev moments.
//
//   theta = sigma W + 1 b^T          (RBM of Sec. I), a [n x N] x [N x M] product on the matrix cores
//   E_loc(s) = sum_bonds [J/4 s_i s_j + [s_i != s_j] J/2 psi(s^{ij})/psi(s)]   (Sec. VI)
//   R(s)     = phi(s)/psi_{n+1}(s)  for the Chebyshev targets of Sec. III
//   mu_n(q)  = < f_q^* beta_n t~_n / psi_gs >                    (Sec. II, App. A)
//
// A pair swap changes theta by Delta_k = -2 s_i (W_ik - W_jk), and
//   cosh(theta_k + Delta_k)/cosh(theta_k) = cosh(Delta_k) + tanh(theta_k) sinh(Delta_k),
// so the amplitude ratio of a bond is a product of M complex factors; each
// lane multiplies its own factors and the wave adds their logarithms.
// Log-amplitude differences between RBMs are summed element by element so
// that the M log 2 constants cancel before any rounding of the total.
#include "device.hpp"
#include "internal.hpp"

namespace crbm {

// ------------------------------------------------------------------ theta GEMM
// theta = sigma W + b on the matrix cores.  sigma = +-1 is exact in BF16, and each
// binary32 W entry is split exactly into three BF16 parts by truncation,
//   W = hi + mid + lo   (8 + 8 + 8 significand bits),
// so three v_mfma_f32_32x32x16_bf16 products give sigma W with exact products and
// FP32 accumulation.  The complex W is a real [N][2M] matrix (re, im interleaved), so the
// output rows are the complex64 theta rows.  Tile: 128 samples x 128 real columns per
// workgroup (4 waves x 32 samples x 4 column blocks), K chunks of 32 sites through LDS.
typedef __attribute__((__vector_size__(8 * sizeof(short)))) short bf16x8_t;
typedef __attribute__((__vector_size__(4 * sizeof(int)))) int i32x4_t;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float floatx16_t;

constexpr int TH_S = 128, TH_C = 128, TH_K = 32;
constexpr int TH_ROW = TH_K * 2 + 16;          // bytes per LDS row (32 bf16 + padding)

__global__ __launch_bounds__(256) void k_theta(const int8_t* __restrict__ sig, long n, int N, int M,
                                                const float2* __restrict__ b, const float2* __restrict__ W,
                                                float2* __restrict__ theta, const double* __restrict__ skip) {
    if (skip && *skip != 0.0) return;     // a converged iterative solve skips the product
    __shared__ __attribute__((aligned(16))) unsigned char s_sig[TH_S * TH_ROW];
    __shared__ __attribute__((aligned(16))) unsigned char s_w[3][TH_C * TH_ROW];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const long s0 = (long)blockIdx.x * TH_S;
    const int c0 = blockIdx.y * TH_C;                 // first real column
    const int C = 2 * M;                              // real columns
    const float* Wf = reinterpret_cast<const float*>(W);
    floatx16_t acc[4];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[cb][v] = 0.f;

    for (int k0 = 0; k0 < N; k0 += TH_K) {
        // sigma tile [128 samples][32 sites] as BF16 (+1 = 0x3F80, -1 = 0xBF80, outside = 0)
        for (int e = tid; e < TH_S * TH_K; e += 256) {
            const int ss = e / TH_K, kk = e % TH_K;
            const long s = s0 + ss;
            const int i = k0 + kk;
            uint16_t v = 0;
            if (s < n && i < N) v = sig[s * N + i] > 0 ? 0x3F80 : 0xBF80;
            *reinterpret_cast<uint16_t*>(s_sig + ss * TH_ROW + kk * 2) = v;
        }
        // W^T tile [128 columns][32 sites], three exact BF16 parts
        for (int e = tid; e < TH_C * TH_K; e += 256) {
            const int kk = e / TH_C, cc = e % TH_C;
            const int i = k0 + kk, c = c0 + cc;
            const float w = (i < N && c < C) ? Wf[(long)i * C + c] : 0.f;
            const uint32_t u = __float_as_uint(w);
            const uint32_t hi = u & 0xFFFF0000u;
            const float r1 = w - __uint_as_float(hi);
            const uint32_t mid = __float_as_uint(r1) & 0xFFFF0000u;
            const float r2 = r1 - __uint_as_float(mid);
            *reinterpret_cast<uint16_t*>(s_w[0] + cc * TH_ROW + kk * 2) = (uint16_t)(hi >> 16);
            *reinterpret_cast<uint16_t*>(s_w[1] + cc * TH_ROW + kk * 2) = (uint16_t)(mid >> 16);
            *reinterpret_cast<uint16_t*>(s_w[2] + cc * TH_ROW + kk * 2) = (uint16_t)(__float_as_uint(r2) >> 16);
        }
        __syncthreads();
#pragma unroll
        for (int kq = 0; kq < TH_K; kq += 16) {
            const int koff = (kq + 8 * (lane >> 5)) * 2;
            const i32x4_t a = *reinterpret_cast<const i32x4_t*>(s_sig + (wave * 32 + (lane & 31)) * TH_ROW + koff);
#pragma unroll
            for (int part = 0; part < 3; ++part)
#pragma unroll
                for (int cb = 0; cb < 4; ++cb) {
                    const i32x4_t bw =
                        *reinterpret_cast<const i32x4_t*>(s_w[part] + (cb * 32 + (lane & 31)) * TH_ROW + koff);
                    acc[cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16((bf16x8_t)a, (bf16x8_t)bw, acc[cb], 0, 0, 0);
                }
        }
        __syncthreads();
    }
    const float* bf = reinterpret_cast<const float*>(b);
    float* out = reinterpret_cast<float*>(theta);
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
        const int c = c0 + cb * 32 + (lane & 31);
        if (c >= C) continue;
        const float bc = bf[c];
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const long s = s0 + wave * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
            if (s < n) out[s * C + c] = acc[cb][v] + bc;
        }
    }
}

hipError_t launch_theta(const int8_t* sig, long n, int N, int M, const float2* b, const float2* W, float2* theta,
                        hipStream_t stream, const double* skip) {
    if (n <= 0) return hipSuccess;
    dim3 grid((unsigned)((n + TH_S - 1) / TH_S), (unsigned)((2 * M + TH_C - 1) / TH_C));
    hipLaunchKernelGGL(k_theta, grid, dim3(256), 0, stream, sig, n, N, M, b, W, theta, skip);
    return hipGetLastError();
}

// ------------------------------------------------------------------ helpers
// f_q(sigma) = N^{-1/2} sum_r exp(-i q.r) sigma_r / 2 over the wave's spins
__device__ __forceinline__ float2 site_phase(int r, int kind, int Lx, double q0, double q1) {
    const int x = kind == 0 ? r : r % Lx;
    const int y = kind == 0 ? 0 : r / Lx;
    const double ph = q0 * x + q1 * y;
    double s, c;
    sincos(ph, &s, &c);
    return make_float2((float)c, (float)-s);
}

__device__ __forceinline__ float2 fq_wave(const WaveSpins& sp, int lane, const Geometry& g, double q0, double q1) {
    float2 acc = make_float2(0.f, 0.f);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int site = q * kWave + lane;
        if (site < g.N) acc = cadd(acc, cscale(site_phase(site, g.kind, g.Lx, q0, q1), 0.5f * (float)sp.s[q]));
    }
    acc = wave_sum(acc);
    return cscale(acc, rsqrtf((float)g.N));
}

// sum_i a_i sigma_i over the wave
__device__ __forceinline__ float2 a_dot_sigma(const float2* a, const WaveSpins& sp, int lane, int N) {
    float2 acc = make_float2(0.f, 0.f);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int site = q * kWave + lane;
        if (site < N) acc = cadd(acc, cscale(a[site], (float)sp.s[q]));
    }
    return acc;
}

// ------------------------------------------------------------------ local estimators
// One wave per sample.  th1/thn/thm: theta of fit / psi_n / psi_{n-1} (precomputed).
template <int E>
__global__ __launch_bounds__(256) void k_local(LocalArgs A, const float2* __restrict__ th1g,
                                               const float2* __restrict__ thng, const float2* __restrict__ thmg) {
    const int lane = threadIdx.x & 63;
    const long s = (long)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (s >= A.n_samples) return;
    const Geometry& g = A.g;
    const int N = g.N, M = g.M;
    WaveSpins sp;
    sp.load(A.samples + s * N, N, lane);

    float2 t1[E], tE[E], TE[E];
    float2 lc1 = make_float2(0.f, 0.f);
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int k = e * kWave + lane;
        t1[e] = (k < M) ? th1g[s * M + k] : make_float2(0.f, 0.f);
    }
    // log psi of fit and tanh theta of fit
    float2 T1[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int k = e * kWave + lane;
        if (k < M) {
            lc1 = cadd(lc1, log2cosh(t1[e]));
            T1[e] = ctanhf(t1[e]);
        } else {
            T1[e] = make_float2(0.f, 0.f);
        }
    }
    const float2 asig1 = a_dot_sigma(A.fit.a, sp, lane, N);
    if (A.logpsi_out) {
        const float2 lp = wave_sum(cadd(lc1, asig1));
        if (lane == 0) A.logpsi_out[s] = lp;
    }
    if (A.tanh_out) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int k = e * kWave + lane;
            if (k < M) A.tanh_out[s * M + k] = T1[e];
        }
    }
    if (A.O_out) {
        float2* row = A.O_out + s * (long)g.P;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int site = q * kWave + lane;
            if (site < N) row[site] = make_float2((float)sp.s[q], 0.f);
        }
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int k = e * kWave + lane;
            if (k < M) row[N + k] = T1[e];
        }
        for (int i = 0; i < N; ++i) {
            const float si = (float)sp.get(i);
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int k = e * kWave + lane;
                if (k < M) row[N + M + (long)i * M + k] = cscale(T1[e], si);
            }
        }
    }
    if (!A.eloc_out && !A.R_out) return;

    // the RBM whose Hamiltonian action is needed
    const RbmView& pe = A.cheb_mode ? A.psn : A.fit;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int k = e * kWave + lane;
        if (A.cheb_mode) {
            tE[e] = (k < M) ? thng[s * M + k] : make_float2(0.f, 0.f);
            TE[e] = (k < M) ? ctanhf(tE[e]) : make_float2(0.f, 0.f);
        } else {
            tE[e] = t1[e];
            TE[e] = T1[e];
        }
    }
    const bool with_fq = A.cheb_mode && A.order == 0;
    // diagonal factor of t_0: f_q (momentum q) or, with local_op, the local S^z_0 = s_0 / 2
    const float2 d0 = !with_fq ? make_float2(1.f, 0.f)
                    : A.local_op ? make_float2(0.5f * (float)sp.get(0), 0.f) : fq_wave(sp, lane, g, A.q0, A.q1);
    const float inv_sqrt_n = rsqrtf((float)N);

    // anti-aligned bonds of this sample, in bond order, compacted into the wave's LDS list
    __shared__ short s_anti[4][kMaxBonds];
    short* lst = s_anti[threadIdx.x >> 6];
    const int8_t* srow = A.samples + s * N;
    int n_anti = 0;
    for (int c0 = 0; c0 < g.n_bonds; c0 += kWave) {
        const int bnd = c0 + lane;
        bool anti = false;
        if (bnd < g.n_bonds) {
            const int2 ij = g.bonds[bnd];
            anti = srow[ij.x] != srow[ij.y];
        }
        const uint64_t m = __ballot(anti);
        if (anti) lst[n_anti + __popcll(m & ((1ull << lane) - 1ull))] = (short)bnd;
        n_anti += __popcll(m);
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

    const float J = (float)g.J;
    // diagonal part: J/4 s_i s_j over all bonds, s_i s_j = -1 on the anti-aligned ones
    const float2 diag = cscale(d0, 0.25f * J * (float)(g.n_bonds - 2 * n_anti));
    float2 acc = make_float2(0.f, 0.f);        // off-diagonal part, on lanes 8 g (group g's bond)
    // Bonds in batches of 8.  Each lane forms its share of a bond's factor product as
    // (log |p|, p/|p|); a reduce-scatter over lane bits 5, 4, 3 then leaves bond b0 + g of the
    // batch on the 8 lanes of group g = lane / 8, which add (multiply) the last 8 shares, so the
    // exponentials and phases of the 8 bonds are evaluated lane-parallel.
    for (int b0 = 0; b0 < n_anti; b0 += 8) {
        float lm[8];
        float2 ph[8];
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            lm[b] = 0.f;
            ph[b] = make_float2(1.f, 0.f);
            if (b0 + b < n_anti) {
                const int bnd = uniform((int)lst[b0 + b]);
                const int i = uniform(g.bonds[bnd].x);
                // Delta_k = -2 s_i D_k with D = W_i - W_j: cosh Delta = cosh 2D, sinh Delta = -s_i sinh 2D,
                // both read from the bond's table
                const float nsi = -(float)sp.get(i);
                const float4* tab = g.bond_tab + (long)bnd * M;
                float2 prod = make_float2(1.f, 0.f);
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const int k = e * kWave + lane;
                    if (k < M) {
                        const float4 q = tab[k];
                        const float2 ts = cmul(TE[e], make_float2(q.z, q.w));
                        prod = cmul(prod, make_float2(fmaf(nsi, ts.x, q.x), fmaf(nsi, ts.y, q.y)));
                    }
                }
                const float n2 = prod.x * prod.x + prod.y * prod.y;
                lm[b] = 0.5f * logf(n2);
                const float inv = n2 > 0.f ? rsqrtf(n2) : 0.f;
                ph[b] = n2 > 0.f ? cscale(prod, inv) : make_float2(1.f, 0.f);
            }
        }
        // reduce-scatter: across lane bit 5 keep 4 of 8 bonds, bit 4 keep 2, bit 3 keep 1
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const bool hi = (lane & 32) != 0;
            const float kl = hi ? lm[t + 4] : lm[t], sl = hi ? lm[t] : lm[t + 4];
            const float2 kp = hi ? ph[t + 4] : ph[t], sp2 = hi ? ph[t] : ph[t + 4];
            lm[t] = kl + __shfl_xor(sl, 32);
            ph[t] = cmul(kp, make_float2(__shfl_xor(sp2.x, 32), __shfl_xor(sp2.y, 32)));
        }
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const bool hi = (lane & 16) != 0;
            const float kl = hi ? lm[t + 2] : lm[t], sl = hi ? lm[t] : lm[t + 2];
            const float2 kp = hi ? ph[t + 2] : ph[t], sp2 = hi ? ph[t] : ph[t + 2];
            lm[t] = kl + __shfl_xor(sl, 16);
            ph[t] = cmul(kp, make_float2(__shfl_xor(sp2.x, 16), __shfl_xor(sp2.y, 16)));
        }
        {
            const bool hi = (lane & 8) != 0;
            const float kl = hi ? lm[1] : lm[0], sl = hi ? lm[0] : lm[1];
            const float2 kp = hi ? ph[1] : ph[0], sp2 = hi ? ph[0] : ph[1];
            lm[0] = kl + __shfl_xor(sl, 8);
            ph[0] = cmul(kp, make_float2(__shfl_xor(sp2.x, 8), __shfl_xor(sp2.y, 8)));
        }
#pragma unroll
        for (int o = 4; o >= 1; o >>= 1) {
            lm[0] += __shfl_xor(lm[0], o);
            ph[0] = cmul(ph[0], make_float2(__shfl_xor(ph[0].x, o), __shfl_xor(ph[0].y, o)));
        }
        const int bb = b0 + (lane >> 3);
        if (bb < n_anti) {
            const int bnd = lst[bb];
            const int2 ij = g.bonds[bnd];
            const int i = ij.x, j = ij.y;
            const float si = (float)srow[i];
            const float m2si = -2.f * si;
            // amplitude ratio psi(s^ij)/psi(s) = exp(sum log|p| + Re da) * (phase) * exp(i Im da)
            const float2 da = cscale(csub(pe.a[i], pe.a[j]), m2si);
            const float ph2 = ph[0].x * ph[0].x + ph[0].y * ph[0].y;
            const float2 u = cscale(ph[0], rsqrtf(ph2));
            float sn, cs;
            sincosf(da.y, &sn, &cs);
            const float2 rho = cscale(cmul(u, make_float2(cs, sn)), expf(lm[0] + da.x));
            float2 d1 = make_float2(1.f, 0.f);
            if (with_fq) {
                if (A.local_op) {
                    // s_0 / 2 after the swap of sites i and j (s_j = -s_i)
                    d1 = make_float2(i == 0 ? -0.5f * si : (j == 0 ? 0.5f * si : d0.x), 0.f);
                } else {
                    // f_q(s^{ij}) = f_q(s) - N^{-1/2} s_i (e^{-iq.r_i} - e^{-iq.r_j})
                    const float2 pd = csub(site_phase(i, g.kind, g.Lx, A.q0, A.q1), site_phase(j, g.kind, g.Lx, A.q0, A.q1));
                    d1 = csub(d0, cscale(pd, inv_sqrt_n * si));
                }
            }
            if ((lane & 7) == 0) acc = cadd(acc, cscale(cmul(d1, rho), 0.5f * J));
        }
    }
    acc = cadd(wave_sum(acc), diag);
    if (A.eloc_out && lane == 0) A.eloc_out[s] = acc;
    if (!A.cheb_mode || !A.R_out) return;

    // R = phi / psi_{n+1}
    const float2 ht = cscale(csub(acc, cmul(make_float2((float)A.E_c, 0.f), d0)), (float)(1.0 / A.W_scale));
    float2 dn = csub(a_dot_sigma(A.psn.a, sp, lane, N), asig1);
#pragma unroll
    for (int e = 0; e < E; ++e)
        if (e * kWave + lane < M) dn = cadd(dn, csub(log2cosh(tE[e]), log2cosh(t1[e])));
    dn = wave_sum(dn);
    const float2 bn = make_float2((float)A.beta_n.x, (float)A.beta_n.y);
    float2 R;
    if (A.order == 0) {
        R = cmul(cmul(bn, ht), cexpf(dn));
    } else {
        float2 dm = csub(a_dot_sigma(A.psm.a, sp, lane, N), asig1);
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int k = e * kWave + lane;
            if (k < M) dm = cadd(dm, csub(log2cosh(thmg[s * M + k]), log2cosh(t1[e])));
        }
        dm = wave_sum(dm);
        const float2 fm = (A.order != 1) ? make_float2(1.f, 0.f)
                        : A.local_op ? make_float2(0.5f * (float)sp.get(0), 0.f) : fq_wave(sp, lane, g, A.q0, A.q1);
        const float2 bm = make_float2((float)A.beta_nm1.x, (float)A.beta_nm1.y);
        R = csub(cscale(cmul(cmul(bn, ht), cexpf(dn)), 2.f), cmul(cmul(bm, fm), cexpf(dm)));
    }
    if (lane == 0) A.R_out[s] = R;
}

// tab[b][k] = (cosh 2D, sinh 2D) with D = W_ik - W_jk for bond b = (i, j); the difference of two
// binary32 values is exact in binary64, and the functions are evaluated there before rounding
__global__ __launch_bounds__(256) void k_bond_table(const int2* __restrict__ bonds, int nb, int M,
                                                    const float2* __restrict__ W, float4* __restrict__ tab) {
    const long idx = (long)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (long)nb * M) return;
    const int b = (int)(idx / M), k = (int)(idx % M);
    const int2 ij = bonds[b];
    const float2 wi = W[(long)ij.x * M + k], wj = W[(long)ij.y * M + k];
    const double x = 2.0 * ((double)wi.x - (double)wj.x), y = 2.0 * ((double)wi.y - (double)wj.y);
    const double ch = cosh(x), sh = sinh(x);
    double sn, cs;
    sincos(y, &sn, &cs);
    tab[idx] = make_float4((float)(ch * cs), (float)(sh * sn), (float)(sh * cs), (float)(ch * sn));
}

hipError_t launch_local_core(const LocalArgs& A, const float2* th1, const float2* thn, const float2* thm,
                             hipStream_t stream) {
    if (A.eloc_out || A.R_out) {
        // the bond factors of the RBM whose Hamiltonian action is taken
        const float2* W = A.cheb_mode ? A.psn.W : A.fit.W;
        const long cnt = (long)A.g.n_bonds * A.g.M;
        hipLaunchKernelGGL(k_bond_table, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, stream, A.g.bonds,
                           A.g.n_bonds, A.g.M, W, A.g.bond_tab);
    }
    const int E = (A.g.M + kWave - 1) / kWave;
    const dim3 grid((unsigned)((A.n_samples + 3) / 4)), block(256);
    switch (E) {
#define CRBM_CASE(e) case e: hipLaunchKernelGGL(k_local<e>, grid, block, 0, stream, A, th1, thn, thm); break;
        CRBM_CASE(1) CRBM_CASE(2) CRBM_CASE(3) CRBM_CASE(4) CRBM_CASE(5) CRBM_CASE(6) CRBM_CASE(7) CRBM_CASE(8)
#undef CRBM_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ------------------------------------------------------------------ moments
// B[n][s] = beta_n exp(log t~_n(s) - log psi_gs(s)) for one order n (one wave per sample).
template <int E>
__global__ __launch_bounds__(256) void k_moment_ratio(int N, int M, const int8_t* __restrict__ sig, long n_s,
                                                      const float2* __restrict__ a_t, const float2* __restrict__ a_g,
                                                      const float2* __restrict__ th_t, const float2* __restrict__ th_g,
                                                      const double2* __restrict__ beta, double2* __restrict__ B) {
    const int lane = threadIdx.x & 63;
    const long s = (long)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (s >= n_s) return;
    WaveSpins sp;
    sp.load(sig + s * N, N, lane);
    float2 d = csub(a_dot_sigma(a_t, sp, lane, N), a_dot_sigma(a_g, sp, lane, N));
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int k = e * kWave + lane;
        if (k < M) d = cadd(d, csub(log2cosh(th_t[s * M + k]), log2cosh(th_g[s * M + k])));
    }
    d = wave_sum(d);
    if (lane == 0) {
        const float2 r = cexpf(d);
        B[s] = zmul(*beta, make_double2((double)r.x, (double)r.y));
    }
}

// f[q][s] = f_q(s) (double) for a chunk of up to 8 momenta, one wave per sample
struct QChunk { double q[8][2]; };

__global__ __launch_bounds__(256) void k_fq(Geometry g, const int8_t* __restrict__ sig, long n_s, QChunk qc, int n_q,
                                            double2* __restrict__ f) {
    const int lane = threadIdx.x & 63;
    const long s = (long)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (s >= n_s) return;
    WaveSpins sp;
    sp.load(sig + s * g.N, g.N, lane);
    const double inv = 1.0 / sqrt((double)g.N);
    for (int iq = 0; iq < n_q; ++iq) {
        double2 acc = make_double2(0.0, 0.0);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int site = q * kWave + lane;
            if (site < g.N) {
                const int x = g.kind == 0 ? site : site % g.Lx;
                const int y = g.kind == 0 ? 0 : site / g.Lx;
                double sn, cs;
                sincos(qc.q[iq][0] * x + qc.q[iq][1] * y, &sn, &cs);
                acc.x += 0.5 * sp.s[q] * cs;
                acc.y -= 0.5 * sp.s[q] * sn;
            }
        }
        acc = wave_sum(acc);
        if (lane == 0) f[(long)iq * n_s + s] = make_double2(acc.x * inv, acc.y * inv);
    }
}

// partial[blk][entry0 + iq*nn] = sum over the block's samples of w conj(f_q) B  (B = f_q when b_is_f)
__global__ __launch_bounds__(256) void k_moment_accum(const double2* __restrict__ f, const double2* __restrict__ B,
                                                      int b_is_f, const double* __restrict__ w, long n_s, int n_q,
                                                      int nn, int entry0, int total, long chunk,
                                                      double2* __restrict__ partial) {
    __shared__ double shx[4], shy[4];
    const long s_begin = (long)blockIdx.x * chunk;
    const long s_end = min(n_s, s_begin + chunk);
    const double wdef = 1.0 / (double)n_s;
    for (int iq = 0; iq < n_q; ++iq) {
        double ax = 0.0, ay = 0.0;
        for (long s = s_begin + threadIdx.x; s < s_end; s += blockDim.x) {
            const double ws = w ? w[s] : wdef;
            const double2 fs = f[(long)iq * n_s + s];
            const double2 t = zconjmul(fs, b_is_f ? fs : B[s]);
            ax += ws * t.x;
            ay += ws * t.y;
        }
        ax = wave_sum(ax);
        ay = wave_sum(ay);
        if ((threadIdx.x & 63) == 0) { shx[threadIdx.x >> 6] = ax; shy[threadIdx.x >> 6] = ay; }
        __syncthreads();
        if (threadIdx.x == 0)
            partial[(long)blockIdx.x * total + entry0 + iq * nn] =
                make_double2(shx[0] + shx[1] + shx[2] + shx[3], shy[0] + shy[1] + shy[2] + shy[3]);
        __syncthreads();
    }
}

__global__ void k_moment_final(const double2* __restrict__ partial, int n_blocks, int total, double2* __restrict__ mu) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    double2 acc = make_double2(0.0, 0.0);
    for (int b = 0; b < n_blocks; ++b) acc = zadd(acc, partial[(long)b * total + idx]);
    mu[idx] = acc;
}

hipError_t launch_moment_ratio(int N, int M, const int8_t* sig, long n_s, const float2* a_t, const float2* a_g,
                               const float2* th_t, const float2* th_g, const double2* beta, double2* B,
                               hipStream_t stream) {
    const int E = (M + kWave - 1) / kWave;
    const dim3 grid((unsigned)((n_s + 3) / 4)), block(256);
    switch (E) {
#define CRBM_CASE(e) case e: hipLaunchKernelGGL(k_moment_ratio<e>, grid, block, 0, stream, N, M, sig, n_s, a_t, a_g, th_t, th_g, beta, B); break;
        CRBM_CASE(1) CRBM_CASE(2) CRBM_CASE(3) CRBM_CASE(4) CRBM_CASE(5) CRBM_CASE(6) CRBM_CASE(7) CRBM_CASE(8)
#undef CRBM_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_fq_chunk(const Geometry& g, const int8_t* sig, long n_s, const double* q_host, int n_q,
                           double2* f, hipStream_t stream) {
    QChunk qc{};
    for (int k = 0; k < n_q && k < 8; ++k) { qc.q[k][0] = q_host[2 * k]; qc.q[k][1] = g.kind == 0 ? 0.0 : q_host[2 * k + 1]; }
    hipLaunchKernelGGL(k_fq, dim3((unsigned)((n_s + 3) / 4)), dim3(256), 0, stream, g, sig, n_s, qc, n_q, f);
    return hipGetLastError();
}

hipError_t launch_moment_accum(const double2* f, const double2* B, int b_is_f, const double* w, long n_s, int n_q,
                               int nn, int entry0, int total, double2* partial, int n_blocks, hipStream_t stream) {
    const long chunk = (n_s + n_blocks - 1) / n_blocks;
    hipLaunchKernelGGL(k_moment_accum, dim3(n_blocks), dim3(256), 0, stream, f, B, b_is_f, w, n_s, n_q, nn, entry0,
                       total, chunk, partial);
    return hipGetLastError();
}

hipError_t launch_moment_final(const double2* partial, int n_blocks, int total, double2* mu, hipStream_t stream) {
    hipLaunchKernelGGL(k_moment_final, dim3((total + 255) / 256), dim3(256), 0, stream, partial, n_blocks, total, mu);
    return hipGetLastError();
}

}  // namespace crbm
