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
// FP32 accumulation.  The B columns of a tile of 64 hidden units are the real and imaginary
// parts of W ordered [Re 0..31 | Im 0..31 | Re 32..63 | Im 32..63], so that both parts of a
// unit end in one lane; W is split into its parts in that order once per RBM (k_wsplit).
// Tile: 128 samples x 128 real columns per workgroup (4 waves x 32 samples x 4 column blocks),
// K chunks of 32 sites through LDS.
typedef __attribute__((__vector_size__(8 * sizeof(short)))) short bf16x8_t;
typedef __attribute__((__vector_size__(4 * sizeof(int)))) int i32x4_t;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float floatx16_t;

constexpr int TH_S = 128, TH_C = 128, TH_K = 32;
constexpr int TH_ROW = TH_K * 2 + 16;          // bytes per LDS row (32 bf16 + padding)

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

// ------------------------------------------------------------------ theta GEMM fused with sum log cosh
// For the moment ratios only the per-sample sums  L(s) = sum_k log cosh theta_k(s)  of an RBM are
// needed, not theta itself.  With both parts of a hidden unit in one lane, each lane forms, row by row,
//   log cosh z = s z + log((1 + w)/2),   s = sign(Re z),  w = exp(-2 s z),  |(1 + w)/2| <= 1,
// keeping s z as a sum and (1 + w)/2 as a product, multiplies the products over the tile's columns
// by a reduce-scatter over the lane bits and takes one complex log per sample row.
//
// The planes of W are [3][Mt 128][Np], Np = N rounded up to TH_K, zero padded; the product's
// workgroups only copy tiles of them.
__global__ __launch_bounds__(256) void k_wsplit(const float2* __restrict__ W, int N, int M, int Np, int Mt,
                                                uint16_t* __restrict__ planes, const double* __restrict__ skip) {
    if (skip && *skip != 0.0) return;     // a converged iterative solve skips the product
    const long rows = (long)Mt * TH_C;
    const long idx = (long)blockIdx.x * 256 + threadIdx.x;
    if (idx >= rows * Np) return;
    const int r = (int)(idx / Np), i = (int)(idx % Np);
    const int rr = r % TH_C, cb = rr / 32;
    const int k = (r / TH_C) * 64 + (cb >> 1) * 32 + rr % 32;
    float w = 0.f;
    if (i < N && k < M) {
        const float2 v = W[(long)i * M + k];
        w = (cb & 1) ? v.y : v.x;
    }
    const uint32_t u = __float_as_uint(w);
    const uint32_t hi = u & 0xFFFF0000u;
    const float r1 = w - __uint_as_float(hi);
    const uint32_t mid = __float_as_uint(r1) & 0xFFFF0000u;
    const float r2 = r1 - __uint_as_float(mid);
    planes[idx] = (uint16_t)(hi >> 16);
    planes[rows * Np + idx] = (uint16_t)(mid >> 16);
    planes[2 * rows * Np + idx] = (uint16_t)(__float_as_uint(r2) >> 16);
}

// combine two partial sums of log cosh: the linear parts add, the bounded factors multiply
__device__ __forceinline__ void lc_join(float2& lin, float2& pr, float2 lin2, float2 pr2) {
    lin = cadd(lin, lin2);
    pr = cmul(pr, pr2);
}

// The tile product: workgroup (x, ct) accumulates sigma[128 x s .. + 128) times the 128 plane rows of
// unit tile ct over all sites, K chunks of TH_K sites through LDS.  Lane l of wave w ends with column
// l % 32 of each 32-column block cb in acc[cb], rows w 32 + 8 (v / 4) + 4 (l / 32) + v % 4.  The kernels
// built on it ask for four waves per SIMD: they then fit in 96 registers with the accumulators among
// them, and four workgroups of 40 KB fill the compute unit's LDS.
__device__ __forceinline__ void theta_tile(const int8_t* __restrict__ sig, long n, int N, int Np,
                                           const uint16_t* __restrict__ planes, long rows, int ct, long s0,
                                           unsigned char* s_sig, unsigned char (*s_w)[TH_C * TH_ROW],
                                           floatx16_t (&acc)[4]) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[cb][v] = 0.f;
    for (int k0 = 0; k0 < Np; k0 += TH_K) {
        for (int e = tid; e < TH_S * TH_K; e += 256) {
            const int ss = e / TH_K, kk = e % TH_K;
            const long sm = s0 + ss;
            const int i = k0 + kk;
            uint16_t v = 0;
            if (sm < n && i < N) v = sig[sm * N + i] > 0 ? 0x3F80 : 0xBF80;
            *reinterpret_cast<uint16_t*>(s_sig + ss * TH_ROW + kk * 2) = v;
        }
        // 3 parts x 128 rows x 32 sites: 16-byte chunks of the planes
        for (int c = tid; c < 3 * TH_C * (TH_K / 8); c += 256) {
            const int part = c / (TH_C * (TH_K / 8)), rem = c % (TH_C * (TH_K / 8));
            const int rr = rem / (TH_K / 8), ch = rem % (TH_K / 8);
            const uint16_t* src = planes + part * rows * Np + ((long)ct * TH_C + rr) * Np + k0 + ch * 8;
            *reinterpret_cast<i32x4_t*>(s_w[part] + rr * TH_ROW + ch * 16) = *reinterpret_cast<const i32x4_t*>(src);
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
}

// theta = sigma W + b, complex64 [n][M]: lane column j holds units 64 ct + j (blocks 0, 1) and
// 64 ct + 32 + j (blocks 2, 3), real and imaginary part together, so 32 lanes store 256 contiguous bytes
__global__ __launch_bounds__(256, 4) void k_theta(const int8_t* __restrict__ sig, long n, int N, int Np, int M,
                                               const float2* __restrict__ b, const uint16_t* __restrict__ planes,
                                               int Mt, float2* __restrict__ theta, const double* __restrict__ skip) {
    if (skip && *skip != 0.0) return;     // a converged iterative solve skips the product
    __shared__ __attribute__((aligned(16))) unsigned char s_sig[TH_S * TH_ROW];
    __shared__ __attribute__((aligned(16))) unsigned char s_w[3][TH_C * TH_ROW];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const long s0 = (long)blockIdx.x * TH_S;
    const int ct = blockIdx.y;
    floatx16_t acc[4];
    theta_tile(sig, n, N, Np, planes, (long)Mt * TH_C, ct, s0, s_sig, s_w, acc);
    const int ku0 = ct * 64 + (lane & 31), ku1 = ku0 + 32;
    const float2 b0 = ku0 < M ? b[ku0] : make_float2(0.f, 0.f);
    const float2 b1 = ku1 < M ? b[ku1] : make_float2(0.f, 0.f);
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const long sm = s0 + wave * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        if (sm >= n) continue;
        if (ku0 < M) theta[sm * M + ku0] = make_float2(acc[0][v] + b0.x, acc[1][v] + b0.y);
        if (ku1 < M) theta[sm * M + ku1] = make_float2(acc[2][v] + b1.x, acc[3][v] + b1.y);
    }
}

hipError_t launch_theta(const int8_t* sig, long n, int N, int M, const float2* b, const float2* W, float2* theta,
                        uint16_t* planes, hipStream_t stream, const double* skip) {
    if (n <= 0) return hipSuccess;
    const int Np = (N + TH_K - 1) / TH_K * TH_K;
    const int Mt = (M + 63) / 64;
    const long cnt = (long)Mt * TH_C * Np;
    hipLaunchKernelGGL(k_wsplit, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, stream, W, N, M, Np, Mt, planes,
                       skip);
    hipLaunchKernelGGL(k_theta, dim3((unsigned)((n + TH_S - 1) / TH_S), (unsigned)Mt), dim3(256), 0, stream, sig, n,
                       N, Np, M, b, planes, Mt, theta, skip);
    return hipGetLastError();
}

// O v of the matrix-free S product without writing G = sigma V_W + v_b: the theta product of V tile by
// tile, each unit's G_sk multiplied by T_sk in the epilogue and the tile's 64 units summed per sample in
// double (products in FP32 widened to double, as a separate pass over G would); a reduce-scatter over
// lane bits 4..0 leaves each row's sum in two lanes.  partial[ct][s] (double2, n per 64-unit tile).
__global__ __launch_bounds__(256, 4) void k_theta_ov(const int8_t* __restrict__ sig, long n, int N, int Np, int M,
                                                  const float2* __restrict__ vb, const uint16_t* __restrict__ planes,
                                                  int Mt, const float2* __restrict__ T, double2* __restrict__ partial,
                                                  const double* __restrict__ skip) {
    if (skip && *skip != 0.0) return;     // a converged iterative solve skips the product
    __shared__ __attribute__((aligned(16))) unsigned char s_sig[TH_S * TH_ROW];
    __shared__ __attribute__((aligned(16))) unsigned char s_w[3][TH_C * TH_ROW];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const long s0 = (long)blockIdx.x * TH_S;
    const int ct = blockIdx.y;
    floatx16_t acc[4];
    theta_tile(sig, n, N, Np, planes, (long)Mt * TH_C, ct, s0, s_sig, s_w, acc);
    const int ku0 = ct * 64 + (lane & 31), ku1 = ku0 + 32;
    const float2 b0 = ku0 < M ? vb[ku0] : make_float2(0.f, 0.f);
    const float2 b1 = ku1 < M ? vb[ku1] : make_float2(0.f, 0.f);
    double px[16], py[16];
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const long sm = s0 + wave * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        px[v] = 0.0;
        py[v] = 0.0;
        if (sm >= n) continue;
        if (ku0 < M) {
            const float2 t = T[sm * M + ku0];
            const float gx = acc[0][v] + b0.x, gy = acc[1][v] + b0.y;
            px[v] += (double)t.x * gx - (double)t.y * gy;
            py[v] += (double)t.x * gy + (double)t.y * gx;
        }
        if (ku1 < M) {
            const float2 t = T[sm * M + ku1];
            const float gx = acc[2][v] + b1.x, gy = acc[3][v] + b1.y;
            px[v] += (double)t.x * gx - (double)t.y * gy;
            py[v] += (double)t.x * gy + (double)t.y * gx;
        }
    }
    // reduce-scatter of the 16 rows over the 32 columns: lane bits 4, 3, 2, 1 halve the rows a lane
    // keeps, bit 0 adds the last pair; the lane ends with row index 8 b4 + 4 b3 + 2 b2 + b1
#pragma unroll
    for (int w = 8, bit = 16; w >= 1; w >>= 1, bit >>= 1) {
        const bool hi = (lane & bit) != 0;
#pragma unroll
        for (int t = 0; t < w; ++t) {
            const double kx = hi ? px[t + w] : px[t], ky = hi ? py[t + w] : py[t];
            const double sx = hi ? px[t] : px[t + w], sy = hi ? py[t] : py[t + w];
            px[t] = kx + __shfl_xor(sx, bit);
            py[t] = ky + __shfl_xor(sy, bit);
        }
    }
    px[0] += __shfl_xor(px[0], 1);
    py[0] += __shfl_xor(py[0], 1);
    if (lane & 1) return;
    const int v = 8 * ((lane >> 4) & 1) + 4 * ((lane >> 3) & 1) + 2 * ((lane >> 2) & 1) + ((lane >> 1) & 1);
    const long sm = s0 + wave * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
    if (sm < n) partial[(long)ct * n + sm] = make_double2(px[0], py[0]);
}

// u[s] = sum over the tiles of partial[ct][s] + sigma_s . v_a: one wave per sample on a bounded grid
// (waves step through the samples), so that the launches a converged solve skips stay cheap
constexpr int kOvFinalBlocks = 4096;
__global__ __launch_bounds__(256) void k_ov_final(int N, long n, int Mt, const int8_t* __restrict__ sig,
                                                  const double2* __restrict__ va, const double2* __restrict__ partial,
                                                  double2* __restrict__ u, const double* __restrict__ skip) {
    if (skip && *skip != 0.0) return;
    const int lane = threadIdx.x & 63;
    for (long s = (long)blockIdx.x * 4 + (threadIdx.x >> 6); s < n; s += (long)gridDim.x * 4) {
        double ax = 0.0, ay = 0.0;
        for (int i = lane; i < N; i += kWave) {
            const double sv = (double)sig[s * N + i];
            ax += sv * va[i].x;
            ay += sv * va[i].y;
        }
        for (int ct = lane; ct < Mt; ct += kWave) {
            const double2 p = partial[(long)ct * n + s];
            ax += p.x;
            ay += p.y;
        }
        ax = wave_sum(ax);
        ay = wave_sum(ay);
        if (lane == 0) u[s] = make_double2(ax, ay);
    }
}

hipError_t launch_theta_ov(const int8_t* sig, long n, int N, int M, const float2* vb, const float2* vW,
                           const double2* va, const float2* T, uint16_t* planes, double2* partial, double2* u,
                           hipStream_t stream, const double* skip) {
    if (n <= 0) return hipSuccess;
    const int Np = (N + TH_K - 1) / TH_K * TH_K;
    const int Mt = (M + 63) / 64;
    const long cnt = (long)Mt * TH_C * Np;
    hipLaunchKernelGGL(k_wsplit, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, stream, vW, N, M, Np, Mt, planes,
                       skip);
    hipLaunchKernelGGL(k_theta_ov, dim3((unsigned)((n + TH_S - 1) / TH_S), (unsigned)Mt), dim3(256), 0, stream, sig,
                       n, N, Np, M, vb, planes, Mt, T, partial, skip);
    const long fb = (n + 3) / 4;
    hipLaunchKernelGGL(k_ov_final, dim3((unsigned)(fb < kOvFinalBlocks ? fb : kOvFinalBlocks)), dim3(256), 0, stream,
                       N, n, Mt, sig, va, partial, u, skip);
    return hipGetLastError();
}

__global__ __launch_bounds__(256, 4) void k_theta_lc(const int8_t* __restrict__ sig, long n, int N, int Np, int M,
                                                  const float2* __restrict__ b, const float2* __restrict__ W,
                                                  const uint16_t* __restrict__ planes, int Mt,
                                                  float2* __restrict__ partial) {
    __shared__ __attribute__((aligned(16))) unsigned char s_sig[TH_S * TH_ROW];
    __shared__ __attribute__((aligned(16))) unsigned char s_w[3][TH_C * TH_ROW];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const long s0 = (long)blockIdx.x * TH_S;
    const int ct = blockIdx.y;                        // 64-unit tile
    floatx16_t acc[4];
    theta_tile(sig, n, N, Np, planes, (long)Mt * TH_C, ct, s0, s_sig, s_w, acc);
    // lane column j = lane % 32: units k0u = 64 ct + j (acc 0, 1) and k1u = k0u + 32 (acc 2, 3)
    const int j = lane & 31;
    const int ku0 = ct * 64 + j, ku1 = ku0 + 32;
    const float2 b0 = ku0 < M ? b[ku0] : make_float2(0.f, 0.f);
    const float2 b1 = ku1 < M ? b[ku1] : make_float2(0.f, 0.f);
    float2 lin[16], pr[16];
    uint32_t poles = 0;   // bit 2 v + h: element (row v, unit h) within the band of a zero of cosh
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        lin[v] = make_float2(0.f, 0.f);
        pr[v] = make_float2(1.f, 0.f);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if ((h == 0 ? ku0 : ku1) >= M) continue;
            const float2 bb = h == 0 ? b0 : b1;
            const float2 z = make_float2(acc[2 * h][v] + bb.x, acc[2 * h + 1][v] + bb.y);
            if (near_pole(z)) poles |= 1u << (2 * v + h);
            else cosh_factor(z, 1.f, lin[v], pr[v]);
        }
    }
    // accumulator element v of lane l is row 8 (v / 4) + 4 (l / 32) + v % 4 of the wave's 32 samples
    while (poles) {
        const int bit = __ffs(poles) - 1;
        poles &= poles - 1;
        const int v = bit >> 1, ku = (bit & 1) ? ku1 : ku0;
        const long row = s0 + wave * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        if (row >= n) continue;
        float2 lcr, thr;
        pole_eval(theta_double(sig + row * N, N, M, ku, b, W), lcr, thr);
#pragma unroll
        for (int vv = 0; vv < 16; ++vv)
            if (vv == v) lin[vv] = cadd(lin[vv], lcr);
    }
    // reduce-scatter of the 16 rows over the 32 columns (lane bits 4..1), then the last pair (bit 0):
    // lane ends with row 8 b4 + 4 b3 + 2 b2 + b1 of its half
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        const bool hi = (lane & 16) != 0;
        const float2 kl = hi ? lin[t + 8] : lin[t], kp = hi ? pr[t + 8] : pr[t];
        const float2 sl = hi ? lin[t] : lin[t + 8], sp = hi ? pr[t] : pr[t + 8];
        lin[t] = kl;
        pr[t] = kp;
        lc_join(lin[t], pr[t], make_float2(__shfl_xor(sl.x, 16), __shfl_xor(sl.y, 16)),
                make_float2(__shfl_xor(sp.x, 16), __shfl_xor(sp.y, 16)));
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const bool hi = (lane & 8) != 0;
        const float2 kl = hi ? lin[t + 4] : lin[t], kp = hi ? pr[t + 4] : pr[t];
        const float2 sl = hi ? lin[t] : lin[t + 4], sp = hi ? pr[t] : pr[t + 4];
        lin[t] = kl;
        pr[t] = kp;
        lc_join(lin[t], pr[t], make_float2(__shfl_xor(sl.x, 8), __shfl_xor(sl.y, 8)),
                make_float2(__shfl_xor(sp.x, 8), __shfl_xor(sp.y, 8)));
    }
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const bool hi = (lane & 4) != 0;
        const float2 kl = hi ? lin[t + 2] : lin[t], kp = hi ? pr[t + 2] : pr[t];
        const float2 sl = hi ? lin[t] : lin[t + 2], sp = hi ? pr[t] : pr[t + 2];
        lin[t] = kl;
        pr[t] = kp;
        lc_join(lin[t], pr[t], make_float2(__shfl_xor(sl.x, 4), __shfl_xor(sl.y, 4)),
                make_float2(__shfl_xor(sp.x, 4), __shfl_xor(sp.y, 4)));
    }
    {
        const bool hi = (lane & 2) != 0;
        const float2 kl = hi ? lin[1] : lin[0], kp = hi ? pr[1] : pr[0];
        const float2 sl = hi ? lin[0] : lin[1], sp = hi ? pr[0] : pr[1];
        lin[0] = kl;
        pr[0] = kp;
        lc_join(lin[0], pr[0], make_float2(__shfl_xor(sl.x, 2), __shfl_xor(sl.y, 2)),
                make_float2(__shfl_xor(sp.x, 2), __shfl_xor(sp.y, 2)));
    }
    lc_join(lin[0], pr[0], make_float2(__shfl_xor(lin[0].x, 1), __shfl_xor(lin[0].y, 1)),
            make_float2(__shfl_xor(pr[0].x, 1), __shfl_xor(pr[0].y, 1)));
    if (lane & 1) return;
    const int v = 8 * ((lane >> 4) & 1) + 4 * ((lane >> 3) & 1) + 2 * ((lane >> 2) & 1) + ((lane >> 1) & 1);
    const long sm = s0 + wave * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
    if (sm >= n) return;
    const float n2 = pr[0].x * pr[0].x + pr[0].y * pr[0].y;
    partial[(long)ct * n + sm] = make_float2(lin[0].x + 0.5f * logf(n2), lin[0].y + atan2f(pr[0].y, pr[0].x));
}

// B[s] = beta exp(a.sigma + sum_tiles partial - Lg[s])  (Lg = NULL: the sums of psi_gs itself go to
// Lg_out instead), one wave per sample; the tile partials and Lg are added in double
__global__ __launch_bounds__(256) void k_lc_final(int N, long n, int Mt, const int8_t* __restrict__ sig,
                                                  const float2* __restrict__ a, const float2* __restrict__ partial,
                                                  const double2* __restrict__ Lg, const double2* __restrict__ beta,
                                                  double2* __restrict__ B, double2* __restrict__ Lg_out) {
    const int lane = threadIdx.x & 63;
    const long s = (long)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (s >= n) return;
    WaveSpins sp;
    sp.load(sig + s * N, N, lane);
    const float2 as = a_dot_sigma(a, sp, lane, N);
    double x = as.x, y = as.y;
    if (lane < Mt) {
        const float2 pt = partial[(long)lane * n + s];
        x += pt.x;
        y += pt.y;
    }
    x = wave_sum(x);
    y = wave_sum(y);
    if (lane != 0) return;
    if (!Lg) {
        Lg_out[s] = make_double2(x, y);
        return;
    }
    const double2 g = Lg[s];
    const double dx = x - g.x, dy = y - g.y;
    const double m = exp(dx);
    double sn, cs;
    sincos(dy, &sn, &cs);
    B[s] = zmul(*beta, make_double2(m * cs, m * sn));
}

hipError_t launch_lc_sums(const int8_t* sig, long n, int N, int M, const float2* a, const float2* b,
                          const float2* W, uint16_t* planes, float2* partial, const double2* Lg,
                          const double2* beta, double2* B, double2* Lg_out, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    const int Np = (N + TH_K - 1) / TH_K * TH_K;
    const int Mt = (M + 63) / 64;
    const long cnt = (long)Mt * TH_C * Np;
    hipLaunchKernelGGL(k_wsplit, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, stream, W, N, M, Np, Mt, planes,
                       nullptr);
    hipLaunchKernelGGL(k_theta_lc, dim3((unsigned)((n + TH_S - 1) / TH_S), (unsigned)Mt), dim3(256), 0, stream, sig,
                       n, N, Np, M, b, W, planes, Mt, partial);
    hipLaunchKernelGGL(k_lc_final, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, stream, N, n, Mt, sig, a, partial,
                       Lg, beta, B, Lg_out);
    return hipGetLastError();
}

// ------------------------------------------------------------------ local estimators
// A wave takes kLocalSpw consecutive samples.  Per sample it evaluates log psi, tanh theta and O
// (lanes over the hidden units) and marks the anti-aligned bonds; then it walks the bonds once:
// a bond's table row is read once and serves every sample of the wave in which the bond is
// anti-aligned.  Each such (sample, bond) pair leaves its per-lane share of the factor product,
// as (log |p|, p/|p|), in a per-wave LDS ring; every 8 pairs a reduce-scatter over lane bits
// 5, 4, 3 gives pair g of the batch to the 8 lanes of group g = lane / 8, which finish it (the
// exponential, the phase of a and the f_q factors) lane-parallel.
constexpr int kLocalSpw = 4;       // samples per wave
constexpr int kRing = 16;          // ring slots per wave: at most 7 + kLocalSpw pairs wait

// Reduce-scatter of 8 bond shares (log |p|, p/|p|) over the wave: across lane bit 5 keep 4 of the 8,
// bit 4 keep 2, bit 3 keep 1, then add (multiply) within the 8 lanes, so that lanes 8 g .. 8 g + 7
// end with the whole of share g in lm[0], ph[0].
__device__ __forceinline__ void reduce_scatter8(float (&lm)[8], float2 (&ph)[8], int lane) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const bool hi = (lane & 32) != 0;
        const float kl = hi ? lm[t + 4] : lm[t], sl = hi ? lm[t] : lm[t + 4];
        const float2 kp = hi ? ph[t + 4] : ph[t], sp = hi ? ph[t] : ph[t + 4];
        lm[t] = kl + __shfl_xor(sl, 32);
        ph[t] = cmul(kp, make_float2(__shfl_xor(sp.x, 32), __shfl_xor(sp.y, 32)));
    }
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const bool hi = (lane & 16) != 0;
        const float kl = hi ? lm[t + 2] : lm[t], sl = hi ? lm[t] : lm[t + 2];
        const float2 kp = hi ? ph[t + 2] : ph[t], sp = hi ? ph[t] : ph[t + 2];
        lm[t] = kl + __shfl_xor(sl, 16);
        ph[t] = cmul(kp, make_float2(__shfl_xor(sp.x, 16), __shfl_xor(sp.y, 16)));
    }
    {
        const bool hi = (lane & 8) != 0;
        const float kl = hi ? lm[1] : lm[0], sl = hi ? lm[0] : lm[1];
        const float2 kp = hi ? ph[1] : ph[0], sp = hi ? ph[0] : ph[1];
        lm[0] = kl + __shfl_xor(sl, 8);
        ph[0] = cmul(kp, make_float2(__shfl_xor(sp.x, 8), __shfl_xor(sp.y, 8)));
    }
#pragma unroll
    for (int o = 4; o >= 1; o >>= 1) {
        lm[0] += __shfl_xor(lm[0], o);
        ph[0] = cmul(ph[0], make_float2(__shfl_xor(ph[0].x, o), __shfl_xor(ph[0].y, o)));
    }
}

// (log |p|, p / |p|) of a lane's share p, from n2 = |p|^2, on the hardware log2 and reciprocal square
// root: n2 is a product of a few factors of modest size, far from the denormal range the library
// forms guard against (p = 0 gives log |p| = -inf and the phase 1).
__device__ __forceinline__ void share_polar(float2 prod, float n2, float& lm, float2& ph) {
    constexpr float kHalfLn2 = 0.34657359027997264f;
    lm = kHalfLn2 * __builtin_amdgcn_logf(n2);
    ph = n2 > 0.f ? cscale(prod, __builtin_amdgcn_rsqf(n2)) : make_float2(1.f, 0.f);
}

// One lane's share of the factor product of an anti-aligned bond (i, j).  With Delta_k = -2 s_i D_k,
// D = W_i - W_j, s_k = sign Re theta_k and w_k = exp(-2 s_k theta_k) (|w_k| <= 1),
//   cosh(theta_k + Delta_k) / cosh theta_k = [exp(s_k Delta_k) + w_k exp(-s_k Delta_k)] / (1 + w_k),
// whose numerator has no cancellation when |Delta| is large (the form cosh Delta + tanh theta sinh Delta
// subtracts two numbers of size exp|Delta| when Re theta and Re Delta have opposite signs).  The bond's
// table row holds (exp 2D, exp -2D); exp(s_k Delta_k) is exp 2D when s_k = -s_i.  The denominators are
// the same for every bond of the sample: qinv = prod 1/(1 + w_k) over this lane's units (each factor in
// [0.58, 1.72] off the zeros of cosh), multiplied into the lane's share so that its logarithm stays the
// logarithm of the lane's part of the ratio; units near a zero of cosh enter a per-sample constant
// instead (bond_term).  neg: bit e set when s_k < 0 for this lane's unit e, flipped for s_i = +1.
template <int E>
__device__ __forceinline__ float2 bond_share(const float4 (&tq)[E], const float2 (&tw)[E], uint32_t neg,
                                             float2 qinv) {
    float2 prod = make_float2(1.f, 0.f);
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const bool sel = ((neg >> e) & 1u) == 0u;
        const float2 X = sel ? make_float2(tq[e].x, tq[e].y) : make_float2(tq[e].z, tq[e].w);
        const float2 Y = sel ? make_float2(tq[e].z, tq[e].w) : make_float2(tq[e].x, tq[e].y);
        const float2 num = make_float2(fmaf(tw[e].x, Y.x, fmaf(-tw[e].y, Y.y, X.x)),
                                       fmaf(tw[e].x, Y.y, fmaf(tw[e].y, Y.x, X.y)));
        prod = cmul(prod, num);
    }
    return cmul(prod, qinv);
}
// the sign word of bond_share for a bond whose first site has spin si
__device__ __forceinline__ uint32_t bond_neg(uint32_t neg, float si) { return si > 0.f ? ~neg : neg; }

// The bond's row of the table for this lane's hidden units (padding lanes give the factor 1).
template <int E>
__device__ __forceinline__ void bond_row(const Geometry& g, int bnd, int lane, float4 (&tq)[E]) {
    const float4* tab = g.bond_tab + (long)bnd * g.M;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int k = e * kWave + lane;
        tq[e] = (k < g.M) ? tab[k] : make_float4(1.f, 0.f, 1.f, 0.f);
    }
}

// The exchange term of bond (i, j) for the sample with spin s_i = si, given the whole factor product
// as (log |p|, phase): J/2 d1 psi(s^ij)/psi(s) with psi(s^ij)/psi(s) = exp(lm + Re da) phase
// exp(i Im da), da = -2 s_i (a_i - a_j) + cq (cq = -sum log(1 + w_k) over the units next to a zero of
// cosh, whose denominators are kept out of the shares), and d1 the diagonal factor of t_0 after the swap.
__device__ __forceinline__ float2 bond_term(const LocalArgs& A, const RbmView& pe, int i, int j, float si, float lm,
                                            float2 ph, float2 d0, float2 cq, bool with_fq, float inv_sqrt_n) {
    const Geometry& g = A.g;
    const float2 da = cadd(cscale(csub(pe.a[i], pe.a[j]), -2.f * si), cq);
    const float2 u = cscale(ph, rsqrtf(ph.x * ph.x + ph.y * ph.y));
    float sn, cs;
    sincosf(da.y, &sn, &cs);
    const float2 rho = cscale(cmul(u, make_float2(cs, sn)), expf(lm + da.x));
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
    return cscale(cmul(d1, rho), 0.5f * (float)g.J);
}

template <int SPW>
__device__ __forceinline__ void local_flush(const LocalArgs& A, const RbmView& pe, int lane, long s0, int done,
                                            int cnt, bool with_fq, float inv_sqrt_n, const float2 (&d0)[SPW],
                                            const float2 (&cq)[SPW], float2 (&acc)[SPW], float (*s_lm)[kWave],
                                            float2 (*s_ph)[kWave], const int* s_item) {
    const Geometry& g = A.g;
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    float lm[8];
    float2 ph[8];
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const int slot = (done + b) & (kRing - 1);
        lm[b] = b < cnt ? s_lm[slot][lane] : 0.f;
        ph[b] = b < cnt ? s_ph[slot][lane] : make_float2(1.f, 0.f);
    }
    reduce_scatter8(lm, ph, lane);
    const int gq = lane >> 3;
    if (gq >= cnt) return;
    const int item = s_item[(done + gq) & (kRing - 1)];
    const int q = item >> 16, bnd = item & 0xFFFF;
    const int2 ij = g.bonds[bnd];
    const float si = (float)A.samples[(s0 + q) * g.N + ij.x];
    float2 d0q = d0[0], cqq = cq[0];
#pragma unroll
    for (int qq = 1; qq < SPW; ++qq) {
        d0q = q == qq ? d0[qq] : d0q;
        cqq = q == qq ? cq[qq] : cqq;
    }
    const float2 c = bond_term(A, pe, ij.x, ij.y, si, lm[0], ph[0], d0q, cqq, with_fq, inv_sqrt_n);
    if ((lane & 7) == 0)
#pragma unroll
        for (int qq = 0; qq < SPW; ++qq)
            if (q == qq) acc[qq] = cadd(acc[qq], c);
}

// This lane's share of sum_k [log cosh theta_k - log cosh phi_k] over its hidden units, theta and phi
// rows of two RBMs (parameters vt, vp) at sample s (spins srow): log cosh z = s z + log((1 + w)/2),
// w = exp(-2 s z), with the linear parts added and the factors of modulus <= 1 multiplied, so that one
// complex log serves E units (the M log 2 of log 2 cosh cancel between the two RBMs); units near a zero
// of cosh are re-evaluated in double and enter the linear part.
template <int E>
__device__ __forceinline__ float2 lc_diff(const float2* __restrict__ th, const float2* __restrict__ ph, long s, int M,
                                          int lane, const RbmView& vt, const RbmView& vp,
                                          const int8_t* __restrict__ srow, int N) {
    float2 lin = make_float2(0.f, 0.f), pt = make_float2(1.f, 0.f), pp = make_float2(1.f, 0.f);
    uint32_t poles = 0;   // bit 2 e + h
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int k = e * kWave + lane;
        if (k >= M) continue;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const float2 z = h == 0 ? th[s * M + k] : ph[s * M + k];
            if (near_pole(z)) poles |= 1u << (2 * e + h);
            else if (h == 0) cosh_factor(z, 1.f, lin, pt);
            else cosh_factor(z, -1.f, lin, pp);
        }
    }
    while (poles) {
        const int bit = __ffs(poles) - 1;
        poles &= poles - 1;
        const int h = bit & 1, k = (bit >> 1) * kWave + lane;
        const RbmView& v = h == 0 ? vt : vp;
        float2 lcr, thr;
        pole_eval(theta_double(srow, N, M, k, v.b, v.W), lcr, thr);
        lin = h == 0 ? cadd(lin, lcr) : csub(lin, lcr);
    }
    // log pt - log pp = log|pt|/|pp| + i arg(pt conj(pp))
    const float2 q = make_float2(pt.x * pp.x + pt.y * pp.y, pt.y * pp.x - pt.x * pp.y);
    const float nt = pt.x * pt.x + pt.y * pt.y, np = pp.x * pp.x + pp.y * pp.y;
    return make_float2(lin.x + 0.5f * (logf(nt) - logf(np)), lin.y + atan2f(q.y, q.x));
}

// One sample of a wave: log psi, tanh theta, O of fit; for the RBM whose Hamiltonian action is taken
// the bond-factor data of bond_share (w_k of this lane's units, their signs neg, the lane's product qinv of
// the denominators and the constant cq of those next to a zero of cosh), the diagonal factor d0 of t_0 and
// the anti-aligned bonds (mask words, count).
template <int E>
__device__ __forceinline__ void local_sample(const LocalArgs& A, const float2* __restrict__ th1g,
                                             const float2* __restrict__ thng, int lane, long s0, int q, int nq,
                                             bool want_local, bool with_fq, int n_words, float2 (&tw)[E],
                                             uint32_t& neg, float2& qinv, float2& cq, float2& d0, int& n_anti,
                                             bool& node, uint64_t* mask) {
    const Geometry& g = A.g;
    const int N = g.N, M = g.M;
    d0 = make_float2(1.f, 0.f);
    n_anti = 0;
    neg = 0u;
    qinv = make_float2(1.f, 0.f);
    cq = make_float2(0.f, 0.f);
    node = false;
#pragma unroll
    for (int e = 0; e < E; ++e) tw[e] = make_float2(0.f, 0.f);
    if (q >= nq) {
        if (lane < n_words) mask[lane] = 0ull;
        return;
    }
    const long s = s0 + q;
    WaveSpins sp;
    sp.load(A.samples + s * N, N, lane);
    float2 t1[E], T1[E];
    float2 lc1 = make_float2(0.f, 0.f);
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int k = e * kWave + lane;
        t1[e] = (k < M) ? th1g[s * M + k] : make_float2(0.f, 0.f);
    }
    // tanh theta of fit, and log psi of fit when asked for; units near a zero of cosh re-evaluated in double
    const int8_t* srow = A.samples + s * N;
    uint32_t poles = 0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int k = e * kWave + lane;
        const bool p = k < M && near_pole(t1[e]);
        poles |= p ? 1u << e : 0u;
        T1[e] = (k < M && !p) ? ctanhf(t1[e]) : make_float2(0.f, 0.f);
        if (A.logpsi_out && k < M && !p) lc1 = cadd(lc1, log2cosh(t1[e]));
    }
    while (poles) {
        const int e = __ffs(poles) - 1;
        poles &= poles - 1;
        float2 lcr, thr;
        pole_eval(theta_double(srow, N, M, e * kWave + lane, A.fit.b, A.fit.W), lcr, thr);
        lc1 = cadd(lc1, make_float2(lcr.x + 0.69314718055994531f, lcr.y));
#pragma unroll
        for (int ee = 0; ee < E; ++ee)
            if (ee == e) T1[ee] = thr;
    }
    if (A.logpsi_out) {
        const float2 lp = wave_sum(cadd(lc1, a_dot_sigma(A.fit.a, sp, lane, N)));
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
        for (int c = 0; c < 4; ++c) {
            const int site = c * kWave + lane;
            if (site < N) row[site] = make_float2((float)sp.s[c], 0.f);
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
    if (!want_local) return;
    // bond-factor data of psi_n (Chebyshev mode) or fit (energy mode): w_k = exp(-2 s_k theta_k) with
    // s_k = sign Re theta_k, qinv = 1 / prod (1 + w_k) over this lane's units, and for the units near a zero
    // of cosh cq = -sum log(1 + w_k) (wave total) with log(1 + w_k) = log 2 - s_k theta_k + log cosh theta_k,
    // theta_k in double
    {
        const float2* thp = A.cheb_mode ? thng : th1g;
        const RbmView& vp = A.cheb_mode ? A.psn : A.fit;
        uint32_t pw = 0;
        float2 q1 = make_float2(1.f, 0.f), cl = make_float2(0.f, 0.f);
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int k = e * kWave + lane;
            if (k >= M) continue;
            const float2 z = thp[s * M + k];
            const float sg = z.x >= 0.f ? 1.f : -1.f;
            neg |= z.x >= 0.f ? 0u : 1u << e;
            const float ex = expf(-2.f * fabsf(z.x));
            const float2 cs = cos_sin(2.f * sg * z.y);
            tw[e] = make_float2(ex * cs.x, -ex * cs.y);
            if (near_pole(z)) pw |= 1u << e;
            else q1 = cmul(q1, make_float2(1.f + tw[e].x, tw[e].y));   // |1 + w| in [0.58, 2] off the band
        }
        node = __ballot(pw != 0u) != 0ull;
        if (lane == 0) g.node_flag[s] = node ? 1 : 0;
        while (pw) {
            const int e = __ffs(pw) - 1;
            pw &= pw - 1;
            const double2 td = theta_double(srow, N, M, e * kWave + lane, vp.b, vp.W);
            float2 lcr, thr;
            pole_eval(td, lcr, thr);
            const float sg = ((neg >> e) & 1u) ? -1.f : 1.f;
            cl = cadd(cl, make_float2(lcr.x + 0.69314718055994531f - sg * (float)td.x, lcr.y - sg * (float)td.y));
        }
        qinv = cdiv(make_float2(1.f, 0.f), q1);
        cq = wave_sum(make_float2(-cl.x, -cl.y));
        cq = make_float2(uniform(cq.x), uniform(cq.y));   // wave-uniform: scalar registers
    }
    // diagonal factor of t_0: f_q (momentum q) or, with local_op, the local S^z_0 = s_0 / 2
    if (with_fq) d0 = A.local_op ? make_float2(0.5f * (float)sp.get(0), 0.f) : fq_wave(sp, lane, g, A.q0, A.q1);
    // anti-aligned bonds of the sample
    for (int c = 0; c < n_words; ++c) {
        const int bnd = c * kWave + lane;
        bool anti = false;
        if (bnd < g.n_bonds) {
            const int2 ij = g.bonds[bnd];
            anti = srow[ij.x] != srow[ij.y];
        }
        const uint64_t m = __ballot(anti);
        if (lane == 0) mask[c] = m;
        n_anti += __popcll(m);
    }
}

// The exchange part of E_loc, sum over anti-aligned bonds of (J/2) d1 psi(s^ij)/psi(s), in double, for a
// sample at which psi (the RBM whose Hamiltonian action is taken) is next to a node (a unit next to a zero
// of cosh): there psi(s) ~ 0 while (H psi)(s) is of the size of E psi(s), so the bond terms are large and
// cancel, which binary32 factors cannot resolve.  theta, every unit factor cosh(theta + Delta)/cosh theta,
// a_i - a_j and f_q are taken in double.  Used by k_local_nodes only, so that the main kernels keep their
// registers and need no stack.
template <int E>
__device__ __forceinline__ double2 exchange_double(const LocalArgs& A, const RbmView& pe, long s, int lane,
                                                const uint64_t* mask, int n_words, bool with_fq) {
    const Geometry& g = A.g;
    const int N = g.N, M = g.M;
    const int8_t* srow = A.samples + s * N;
    double2 th[E], lc[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int k = e * kWave + lane;
        th[e] = k < M ? theta_double(srow, N, M, k, pe.b, pe.W) : make_double2(0.0, 0.0);
        lc[e] = k < M ? log_cosh_double(th[e]) : make_double2(0.0, 0.0);
    }
    const double inv_sqrt_n = 1.0 / sqrt((double)N);
    auto phase = [&](int r) {
        const int x = g.kind == 0 ? r : r % g.Lx, y = g.kind == 0 ? 0 : r / g.Lx;
        double sn, cs;
        sincos(A.q0 * x + A.q1 * y, &sn, &cs);
        return make_double2(cs, -sn);
    };
    double2 fq = make_double2(0.0, 0.0);
    if (with_fq && !A.local_op) {
        for (int r = lane; r < N; r += kWave) {
            const double2 p = phase(r);
            fq.x += 0.5 * srow[r] * p.x;
            fq.y += 0.5 * srow[r] * p.y;
        }
        fq = wave_sum(fq);
        fq = make_double2(fq.x * inv_sqrt_n, fq.y * inv_sqrt_n);
    }
    double2 acc = make_double2(0.0, 0.0);
    for (int c = 0; c < n_words; ++c) {
        uint64_t m = mask[c];
        while (m) {
            const int bnd = c * kWave + __builtin_ctzll(m);
            m &= m - 1ull;
            const int2 ij = g.bonds[bnd];
            const double si = (double)srow[ij.x];
            double2 d = make_double2(0.0, 0.0);
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int k = e * kWave + lane;
                if (k >= M) continue;
                const float2 wi = pe.W[(long)ij.x * M + k], wj = pe.W[(long)ij.y * M + k];
                const double2 z = make_double2(th[e].x - 2.0 * si * ((double)wi.x - (double)wj.x),
                                               th[e].y - 2.0 * si * ((double)wi.y - (double)wj.y));
                const double2 l2 = log_cosh_double(z);
                d.x += l2.x - lc[e].x;
                d.y += l2.y - lc[e].y;
            }
            d = wave_sum(d);
            const float2 ai = pe.a[ij.x], aj = pe.a[ij.y];
            d.x -= 2.0 * si * ((double)ai.x - (double)aj.x);
            d.y -= 2.0 * si * ((double)ai.y - (double)aj.y);
            const double mag = exp(d.x);
            double sn, cs;
            sincos(d.y, &sn, &cs);
            double2 t = make_double2(0.5 * g.J * mag * cs, 0.5 * g.J * mag * sn);
            if (with_fq) {
                double2 d1;
                if (A.local_op) {
                    d1 = make_double2(ij.x == 0 ? -0.5 * si : (ij.y == 0 ? 0.5 * si : 0.5 * srow[0]), 0.0);
                } else {
                    const double2 pi_ = phase(ij.x), pj = phase(ij.y);
                    d1 = make_double2(fq.x - inv_sqrt_n * si * (pi_.x - pj.x), fq.y - inv_sqrt_n * si * (pi_.y - pj.y));
                }
                t = zmul(d1, t);
            }
            acc = zadd(acc, t);
        }
    }
    return acc;
}

// One sample's local energy (J/4 s_i s_j over all bonds plus the exchange part in acc, already summed
// over the lanes that hold it, or formed in double at a node of psi) and, in Chebyshev mode, R = phi / psi_{n+1}.
template <int E, bool NODE>
__device__ __forceinline__ void local_finish(const LocalArgs& A, const float2* __restrict__ th1g,
                                             const float2* __restrict__ thng, const float2* __restrict__ thmg,
                                             int lane, long s, float2 acc, float2 d0, int n_anti,
                                             const uint64_t* mask, int n_words) {
    const Geometry& g = A.g;
    const int N = g.N, M = g.M;
    const float J = (float)g.J;
    float2 exch;
    if (NODE) {
        const double2 x = exchange_double<E>(A, A.cheb_mode ? A.psn : A.fit, s, lane, mask, n_words,
                                             A.cheb_mode && A.order == 0);
        exch = make_float2((float)x.x, (float)x.y);
    } else {
        exch = wave_sum(acc);
    }
    const float2 eloc = cadd(exch, cscale(d0, 0.25f * J * (float)(g.n_bonds - 2 * n_anti)));
    if (A.eloc_out && lane == 0) A.eloc_out[s] = eloc;
    if (!A.cheb_mode || !A.R_out) return;
    WaveSpins sp;
    sp.load(A.samples + s * N, N, lane);
    const float2 asig1 = a_dot_sigma(A.fit.a, sp, lane, N);
    const float2 ht = cscale(csub(eloc, cmul(make_float2((float)A.E_c, 0.f), d0)), (float)(1.0 / A.W_scale));
    const int8_t* srow = A.samples + s * N;
    float2 dn = cadd(csub(a_dot_sigma(A.psn.a, sp, lane, N), asig1),
                     lc_diff<E>(thng, th1g, s, M, lane, A.psn, A.fit, srow, N));
    dn = wave_sum(dn);
    // beta enters through its logarithm, added to the log-amplitude difference before the exponential, so
    // that neither a small beta nor a large ratio of unnormalised states leaves the binary32 range on its own
    float2 R;
    if (A.order == 0) {
        R = cmul(ht, cexpf(cadd(dn, A.lbeta_n)));
    } else {
        float2 dm = cadd(csub(a_dot_sigma(A.psm.a, sp, lane, N), asig1),
                         lc_diff<E>(thmg, th1g, s, M, lane, A.psm, A.fit, srow, N));
        dm = wave_sum(dm);
        const float2 fm = (A.order != 1) ? make_float2(1.f, 0.f)
                        : A.local_op ? make_float2(0.5f * (float)sp.get(0), 0.f) : fq_wave(sp, lane, g, A.q0, A.q1);
        R = csub(cscale(cmul(ht, cexpf(cadd(dn, A.lbeta_n))), 2.f), cmul(fm, cexpf(cadd(dm, A.lbeta_nm1))));
    }
    if (lane == 0) A.R_out[s] = R;
}

// Three waves per SIMD up to 7 x 64 hidden units: E = 6 and 7 then spill 44 and 80 bytes per lane, and
// the third wave still makes the bond walk 15% faster at E = 7; E = 8 keeps two waves (with three, its
// 128-byte spill made it 2% slower).
template <int E>
__global__ __launch_bounds__(256, E <= 7 ? 3 : 2) void k_local(LocalArgs A, const float2* __restrict__ th1g,
                                               const float2* __restrict__ thng, const float2* __restrict__ thmg) {
    constexpr int SPW = kLocalSpw;
    __shared__ uint64_t s_mask[4][SPW][kMaxBonds / 64];
    __shared__ float s_lm[4][kRing][kWave];
    __shared__ float2 s_ph[4][kRing][kWave];
    __shared__ int s_item[4][kRing];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const long s0 = ((long)blockIdx.x * 4 + wv) * SPW;
    if (s0 >= A.n_samples) return;
    const Geometry& g = A.g;
    const int N = g.N, M = g.M;
    const int nq = (int)(A.n_samples - s0 < SPW ? A.n_samples - s0 : SPW);
    const bool want_local = A.eloc_out || A.R_out;
    const bool with_fq = A.cheb_mode && A.order == 0;
    // the RBM whose Hamiltonian action is needed
    const RbmView& pe = A.cheb_mode ? A.psn : A.fit;
    const int n_words = (g.n_bonds + 63) / 64;

    float2 TW[SPW][E];
    uint32_t NEG[SPW];
    float2 QI[SPW], CQ[SPW];
    bool NODE[SPW];
    float2 d0[SPW];
    int n_anti[SPW];
    static_assert(SPW == 4, "the per-sample calls below are written out for 4 samples");
    local_sample<E>(A, th1g, thng, lane, s0, 0, nq, want_local, with_fq, n_words, TW[0], NEG[0], QI[0], CQ[0], d0[0],
                    n_anti[0], NODE[0],
                    s_mask[wv][0]);
    local_sample<E>(A, th1g, thng, lane, s0, 1, nq, want_local, with_fq, n_words, TW[1], NEG[1], QI[1], CQ[1], d0[1],
                    n_anti[1], NODE[1],
                    s_mask[wv][1]);
    local_sample<E>(A, th1g, thng, lane, s0, 2, nq, want_local, with_fq, n_words, TW[2], NEG[2], QI[2], CQ[2], d0[2],
                    n_anti[2], NODE[2],
                    s_mask[wv][2]);
    local_sample<E>(A, th1g, thng, lane, s0, 3, nq, want_local, with_fq, n_words, TW[3], NEG[3], QI[3], CQ[3], d0[3],
                    n_anti[3], NODE[3],
                    s_mask[wv][3]);
    if (!want_local) return;
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

    const float inv_sqrt_n = rsqrtf((float)N);
    float2 acc[SPW];
#pragma unroll
    for (int q = 0; q < SPW; ++q) acc[q] = make_float2(0.f, 0.f);
    int pushed = 0, done = 0;
    for (int c = 0; c < n_words; ++c) {
        uint64_t mk[SPW];
        uint64_t any = 0ull;
#pragma unroll
        for (int q = 0; q < SPW; ++q) {
            mk[q] = s_mask[wv][q][c];
            any |= mk[q];
        }
        while (any) {
            const int bit = __builtin_ctzll(any);
            any &= any - 1ull;
            const int bnd = c * kWave + bit;
            const int i = uniform(g.bonds[bnd].x);
            float4 tq[E];
            bond_row<E>(g, bnd, lane, tq);
#pragma unroll
            for (int q = 0; q < SPW; ++q) {
                if (!((mk[q] >> bit) & 1ull)) continue;
                const float2 prod =
                    bond_share<E>(tq, TW[q], bond_neg(NEG[q], (float)A.samples[(s0 + q) * N + i]), QI[q]);
                const int slot = pushed & (kRing - 1);
                float lmv;
                float2 phv;
                share_polar(prod, prod.x * prod.x + prod.y * prod.y, lmv, phv);
                s_lm[wv][slot][lane] = lmv;
                s_ph[wv][slot][lane] = phv;
                if (lane == 0) s_item[wv][slot] = (q << 16) | bnd;
                ++pushed;
            }
            if (pushed - done >= 8) {
                local_flush<SPW>(A, pe, lane, s0, done, 8, with_fq, inv_sqrt_n, d0, CQ, acc, s_lm[wv], s_ph[wv],
                                 s_item[wv]);
                done += 8;
            }
        }
    }
    while (done < pushed) {
        const int cnt = pushed - done < 8 ? pushed - done : 8;
        local_flush<SPW>(A, pe, lane, s0, done, cnt, with_fq, inv_sqrt_n, d0, CQ, acc, s_lm[wv], s_ph[wv],
                         s_item[wv]);
        done += cnt;
    }

    local_finish<E, false>(A, th1g, thng, thmg, lane, s0, acc[0], d0[0], n_anti[0], s_mask[wv][0], n_words);
    if (nq > 1) local_finish<E, false>(A, th1g, thng, thmg, lane, s0 + 1, acc[1], d0[1], n_anti[1], s_mask[wv][1], n_words);
    if (nq > 2) local_finish<E, false>(A, th1g, thng, thmg, lane, s0 + 2, acc[2], d0[2], n_anti[2], s_mask[wv][2], n_words);
    if (nq > 3) local_finish<E, false>(A, th1g, thng, thmg, lane, s0 + 3, acc[3], d0[3], n_anti[3], s_mask[wv][3], n_words);
}

// Narrow RBMs (M <= 3 x 64): one sample per wave.  With few hidden units per lane the bookkeeping of
// the bond-major walk costs more than the table reads it saves, so each wave walks its own sample's
// anti-aligned bonds in batches of 8 with the shares kept in registers.  Five waves per SIMD: the
// kernel fits in 96 registers without spilling, and the walk's table reads want the extra wave.
template <int E>
__global__ __launch_bounds__(256, 5) void k_local_one(LocalArgs A, const float2* __restrict__ th1g,
                                                   const float2* __restrict__ thng, const float2* __restrict__ thmg) {
    __shared__ uint64_t s_mask[4][kMaxBonds / 64];
    __shared__ short s_anti[4][kMaxBonds];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const long s = (long)blockIdx.x * 4 + wv;
    if (s >= A.n_samples) return;
    const Geometry& g = A.g;
    const bool want_local = A.eloc_out || A.R_out;
    const bool with_fq = A.cheb_mode && A.order == 0;
    const RbmView& pe = A.cheb_mode ? A.psn : A.fit;
    const int n_words = (g.n_bonds + 63) / 64;
    float2 TW[E];
    uint32_t neg;
    float2 qinv, cq;
    float2 d0;
    int n_anti;
    bool node;
    local_sample<E>(A, th1g, thng, lane, s, 0, 1, want_local, with_fq, n_words, TW, neg, qinv, cq, d0, n_anti, node,
                    s_mask[wv]);
    if (!want_local) return;
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // the anti-aligned bonds in bond order
    short* lst = s_anti[wv];
    int base = 0;
    for (int c = 0; c < n_words; ++c) {
        const uint64_t m = s_mask[wv][c];
        if ((m >> lane) & 1ull) lst[base + __popcll(m & ((1ull << lane) - 1ull))] = (short)(c * kWave + lane);
        base += __popcll(m);
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const float inv_sqrt_n = rsqrtf((float)g.N);
    const int8_t* srow = A.samples + s * g.N;
    float2 acc = make_float2(0.f, 0.f);
    for (int b0 = 0; b0 < n_anti; b0 += 8) {
        float lm[8];
        float2 ph[8];
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            lm[b] = 0.f;
            ph[b] = make_float2(1.f, 0.f);
            if (b0 + b < n_anti) {
                const int bnd = uniform((int)lst[b0 + b]);
                float4 tq[E];
                bond_row<E>(g, bnd, lane, tq);
                const float2 prod = bond_share<E>(tq, TW, bond_neg(neg, (float)srow[uniform(g.bonds[bnd].x)]), qinv);
                share_polar(prod, prod.x * prod.x + prod.y * prod.y, lm[b], ph[b]);
            }
        }
        reduce_scatter8(lm, ph, lane);
        const int bb = b0 + (lane >> 3);
        if (bb < n_anti) {
            const int2 ij = g.bonds[lst[bb]];
            const float2 c = bond_term(A, pe, ij.x, ij.y, (float)srow[ij.x], lm[0], ph[0], d0, cq, with_fq, inv_sqrt_n);
            if ((lane & 7) == 0) acc = cadd(acc, c);
        }
    }
    local_finish<E, false>(A, th1g, thng, thmg, lane, s, acc, d0, n_anti, s_mask[wv], n_words);
}

// Samples at which the local-energy RBM is next to a node (flagged by k_local / k_local_one): E_loc with
// the exchange sum in double (exchange_double) and, in Chebyshev mode, R, overwriting the binary32 values
// of the main kernel.  One wave per sample; unflagged samples return at once.
template <int E>
__global__ __launch_bounds__(256) void k_local_nodes(LocalArgs A, const float2* __restrict__ th1g,
                                                     const float2* __restrict__ thng, const float2* __restrict__ thmg) {
    __shared__ uint64_t s_mask[4][kMaxBonds / 64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const long s = (long)blockIdx.x * 4 + wv;
    if (s >= A.n_samples) return;
    const Geometry& g = A.g;
    if (!g.node_flag[s]) return;
    const int8_t* srow = A.samples + s * g.N;
    const int n_words = (g.n_bonds + 63) / 64;
    int n_anti = 0;
    for (int c = 0; c < n_words; ++c) {
        const int bnd = c * kWave + lane;
        bool anti = false;
        if (bnd < g.n_bonds) {
            const int2 ij = g.bonds[bnd];
            anti = srow[ij.x] != srow[ij.y];
        }
        const uint64_t m = __ballot(anti);
        if (lane == 0) s_mask[wv][c] = m;
        n_anti += __popcll(m);
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    float2 d0 = make_float2(1.f, 0.f);
    if (A.cheb_mode && A.order == 0) {
        WaveSpins sp;
        sp.load(srow, g.N, lane);
        d0 = A.local_op ? make_float2(0.5f * (float)sp.get(0), 0.f) : fq_wave(sp, lane, g, A.q0, A.q1);
    }
    local_finish<E, true>(A, th1g, thng, thmg, lane, s, make_float2(0.f, 0.f), d0, n_anti, s_mask[wv], n_words);
}

// (exp 2D, exp -2D) per bond and hidden unit, D = W_i - W_j, from the binary32 weights in double
__global__ __launch_bounds__(256) void k_bond_table(const int2* __restrict__ bonds, int nb, int M,
                                                    const float2* __restrict__ W, float4* __restrict__ tab) {
    const long idx = (long)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (long)nb * M) return;
    const int b = (int)(idx / M), k = (int)(idx % M);
    const int2 ij = bonds[b];
    const float2 wi = W[(long)ij.x * M + k], wj = W[(long)ij.y * M + k];
    const double x = 2.0 * ((double)wi.x - (double)wj.x), y = 2.0 * ((double)wi.y - (double)wj.y);
    const double ep = exp(x), em = exp(-x);
    double sn, cs;
    sincos(y, &sn, &cs);
    tab[idx] = make_float4((float)(ep * cs), (float)(ep * sn), (float)(em * cs), (float)(-em * sn));
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
    const dim3 block(256);
    const dim3 grid1((unsigned)((A.n_samples + 3) / 4));
    const long per_block = 4L * kLocalSpw;
    const dim3 grid4((unsigned)((A.n_samples + per_block - 1) / per_block));
    switch (E) {
#define CRBM_ONE(e) case e: hipLaunchKernelGGL(k_local_one<e>, grid1, block, 0, stream, A, th1, thn, thm); break;
#define CRBM_BM(e) case e: hipLaunchKernelGGL(k_local<e>, grid4, block, 0, stream, A, th1, thn, thm); break;
        CRBM_ONE(1) CRBM_ONE(2) CRBM_ONE(3) CRBM_BM(4) CRBM_BM(5) CRBM_BM(6) CRBM_BM(7) CRBM_BM(8)
#undef CRBM_ONE
#undef CRBM_BM
        default: return hipErrorInvalidValue;
    }
    if (A.eloc_out || A.R_out) {
        switch (E) {
#define CRBM_NODES(e) case e: hipLaunchKernelGGL(k_local_nodes<e>, grid1, block, 0, stream, A, th1, thn, thm); break;
            CRBM_NODES(1) CRBM_NODES(2) CRBM_NODES(3) CRBM_NODES(4) CRBM_NODES(5) CRBM_NODES(6) CRBM_NODES(7)
            CRBM_NODES(8)
#undef CRBM_NODES
            default: return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

// ------------------------------------------------------------------ moments
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
