// Natural-gradient (stochastic reconfiguration) step of Sec. III on the GPU.
//
// With the extended index sets i in [0, N] and j in [0, M], where sigma~_N = 1
// and T~_M = 1, every log-derivative is a product O_(i,j)(s) = sigma~_si T~_sj:
// (i < N, j = M) is O_{a_i} = sigma_i, (i = N, j < M) is O_{b_j} = tanh theta_j
// and (i < N, j < M) is O_{W_ij}.  Every P-vector contraction over samples,
//   out_(i,j) = sum_s sigma~_si conj(T~_sj) c_s,
// is then one [(N+1) x n] x [n x (M+1)] product with a per-sample complex
// coefficient c_s:  <O>^* (c = w), <O^* R> (c = w R), the matrix-free
// S v (c = w u, u = O v) and the fidelity gradient (c = 2(1-R) conj(R)/n).
// Partial sums run in FP32 over a chunk of samples and in FP64 across chunks.
#include <float.h>

#include <algorithm>

#include "../../include/chebrbm.h"
#include "device.hpp"
#include "internal.hpp"

namespace crbm {


// device scalar slots (SC_RR and SC_RR1 hold r^H r of the even and odd CG iterations; SC_WSUM the sum of the
// sample weights)
enum {
    SC_RM_RE = 0, SC_RM_IM, SC_R2, SC_GAMMA, SC_GCOT, SC_COEF,
    SC_RR = 8, SC_PAP, SC_RR1, SC_WSUM, SC_FF, SC_DONE, SC_ITERS, SC_FLAGS, SC_RESID, SC_XX,
    SC_COUNT = 32
};

// ------------------------------------------------------------------ P-index <-> (i, j)
__device__ __forceinline__ void p_to_ij(long k, int N, int M, int& i, int& j) {
    if (k < N) { i = (int)k; j = M; }
    else if (k < N + M) { i = N; j = (int)(k - N); }
    else { const long r = k - N - M; i = (int)(r / M); j = (int)(r % M); }
}
__device__ __forceinline__ long ij_to_p(int i, int j, int N, int M) {
    if (j == M) return i;                 // i < N
    if (i == N) return (long)N + j;
    return (long)N + M + (long)i * M + j;
}

// ------------------------------------------------------------------ scalar reductions
// red[2 blk] = (sum w Re R, sum w Im R), red[2 blk + 1] = (sum w |R|^2, sum w)
__global__ __launch_bounds__(256) void k_r_moments(const float2* __restrict__ R, const double* __restrict__ w, long n,
                                                   double2* __restrict__ red) {
    __shared__ double sh[4][4];
    double rx = 0, ry = 0, r2 = 0, ws_sum = 0;
    const double wdef = 1.0 / (double)n;
    for (long s = (long)blockIdx.x * 256 + threadIdx.x; s < n; s += (long)gridDim.x * 256) {
        const double ws = w ? w[s] : wdef;
        const double x = R[s].x, y = R[s].y;
        rx += ws * x; ry += ws * y; r2 += ws * (x * x + y * y); ws_sum += ws;
    }
    rx = wave_sum(rx); ry = wave_sum(ry); r2 = wave_sum(r2); ws_sum = wave_sum(ws_sum);
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) { sh[0][wv] = rx; sh[1][wv] = ry; sh[2][wv] = r2; sh[3][wv] = ws_sum; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0, b = 0, c = 0, d = 0;
        for (int k = 0; k < 4; ++k) { a += sh[0][k]; b += sh[1][k]; c += sh[2][k]; d += sh[3][k]; }
        red[2 * blockIdx.x] = make_double2(a, b);
        red[2 * blockIdx.x + 1] = make_double2(c, d);
    }
}

// Fit mode (0): gamma = arccos sqrt(|<R>|^2/<|R|^2>) and the force scale dgamma gamma cot gamma.
// Energy mode (1): R holds E_loc; the SC_GAMMA slot takes the variance <|E|^2> - |<E>|^2 and the
// force scale is -lr (passed as dgamma).
__global__ void k_r_final(const double2* __restrict__ red, int n_blocks, double dgamma, int mode,
                          double* __restrict__ sc) {
    if (threadIdx.x != 0) return;
    double a = 0, b = 0, c = 0, d = 0;
    for (int k = 0; k < n_blocks; ++k) {
        a += red[2 * k].x; b += red[2 * k].y; c += red[2 * k + 1].x; d += red[2 * k + 1].y;
    }
    sc[SC_RM_RE] = a; sc[SC_RM_IM] = b; sc[SC_R2] = c;
    for (int k = SC_RR; k < SC_COUNT; ++k) sc[k] = 0.0;
    sc[SC_WSUM] = d;
    if (mode == 1) {
        sc[SC_GAMMA] = c - (a * a + b * b);
        sc[SC_GCOT] = 1.0;
        sc[SC_COEF] = dgamma;
        if (!isfinite(a) || !isfinite(b) || !isfinite(c)) sc[SC_FLAGS] = CRBM_FLAG_NONFINITE;
        return;
    }
    const double ratio = (a * a + b * b) / c;
    const double gamma = acos(fmin(1.0, sqrt(ratio)));
    const double gcot = (gamma < 1e-4) ? 1.0 - gamma * gamma / 3.0 : gamma / tan(gamma);
    sc[SC_GAMMA] = gamma; sc[SC_GCOT] = gcot; sc[SC_COEF] = dgamma * gcot;
    if (!(c > 0.0) || !isfinite(a) || !isfinite(b) || !isfinite(c)) sc[SC_FLAGS] = CRBM_FLAG_NONFINITE;
}

// gamma and beta = <R> of the fit as it stands (Sec. III: beta is taken once the steps are done):
// out = {gamma, Re <R>, Im <R>, <|R|^2>, flags}
__global__ void k_fit_stats(const double2* __restrict__ red, int n_blocks, double* __restrict__ out) {
    if (threadIdx.x != 0) return;
    double a = 0, b = 0, c = 0;
    for (int k = 0; k < n_blocks; ++k) { a += red[2 * k].x; b += red[2 * k].y; c += red[2 * k + 1].x; }
    const double gamma = acos(fmin(1.0, sqrt((a * a + b * b) / c)));
    out[0] = gamma;
    out[1] = a;
    out[2] = b;
    out[3] = c;
    out[4] = (!(c > 0.0) || !isfinite(a) || !isfinite(b) || !isfinite(c)) ? (double)CRBM_FLAG_NONFINITE : 0.0;
}

// Exact-enumeration weights p(s) = |psi_s|^2 / sum_s' |psi_s'|^2 = exp(2 Re log psi_s - LSE) (the sampling
// distribution of Sec. III with every configuration listed once).  Pass 1: per block the largest
// 2 Re log psi and the sum of exp(2 Re log psi - that largest value).  Pass 2: every block merges the
// partials in block order (the same result in every block) and writes its share of the weights.
constexpr int kLseBlocks = kLseParts;
__global__ __launch_bounds__(256) void k_lse_partial(const float2* __restrict__ lp, long n, double2* __restrict__ part) {
    __shared__ double sh[4];
    double mx = -INFINITY;
    for (long s = (long)blockIdx.x * 256 + threadIdx.x; s < n; s += (long)gridDim.x * 256)
        mx = fmax(mx, 2.0 * (double)lp[s].x);
    for (int o = 32; o >= 1; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, kWave));
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = mx;
    __syncthreads();
    mx = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
    double acc = 0.0;
    if (mx > -INFINITY)
        for (long s = (long)blockIdx.x * 256 + threadIdx.x; s < n; s += (long)gridDim.x * 256)
            acc += exp(2.0 * (double)lp[s].x - mx);
    acc = wave_sum(acc);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = make_double2(mx, sh[0] + sh[1] + sh[2] + sh[3]);
}
__global__ __launch_bounds__(256) void k_lse_weights(const float2* __restrict__ lp, long n,
                                                     const double2* __restrict__ part, int n_part,
                                                     double* __restrict__ w) {
    __shared__ double lse;
    if (threadIdx.x == 0) {
        double mx = -INFINITY;
        for (int k = 0; k < n_part; ++k) mx = fmax(mx, part[k].x);
        double z = 0.0;
        for (int k = 0; k < n_part; ++k)
            if (part[k].x > -INFINITY) z += part[k].y * exp(part[k].x - mx);
        lse = mx + log(z);   // NaN or infinite when no amplitude is finite and non-zero
    }
    __syncthreads();
    const double L = lse;
    for (long s = (long)blockIdx.x * 256 + threadIdx.x; s < n; s += (long)gridDim.x * 256)
        w[s] = exp(2.0 * (double)lp[s].x - L);
}

hipError_t launch_fit_stats(const float2* R, const double* w, long n, double2* red, double* out, hipStream_t stream) {
    const int nb = 256;
    hipLaunchKernelGGL(k_r_moments, dim3(nb), dim3(256), 0, stream, R, w, n, red);
    hipLaunchKernelGGL(k_fit_stats, dim3(1), dim3(64), 0, stream, red, nb, out);
    return hipGetLastError();
}

hipError_t launch_enum_weights(const float2* lp, long n, double2* part, double* w, hipStream_t stream) {
    hipLaunchKernelGGL(k_lse_partial, dim3(kLseBlocks), dim3(256), 0, stream, lp, n, part);
    const unsigned nb = (unsigned)std::min<long>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(k_lse_weights, dim3(nb), dim3(256), 0, stream, lp, n, part, kLseBlocks, w);
    return hipGetLastError();
}

// ------------------------------------------------------------------ O^H c contraction
// out_c[i][j] = sum_s sigma~_i(s) y_c(s, j) with y_c(s, j) = c_c(s) conj(t~_j(s)), sigma~_N = 1 and
// t~_M = 1: per coefficient a real (N+1) x n by n x (M+1) complex product (rows i < N are the a
// parameters' O, row N the b parameters', the rest W's, up to conjugation and the sample weights).
// On the matrix cores with v_mfma_f32_32x32x2f32, so products and sums stay FP32 as on the vector
// units.  A workgroup (4 waves) owns 128 extended sites x 32 extended hidden units and a run of
// sample chunks; per 32-sample tile it stages sigma~ as floats [site][sample] and y as [c][Re/Im][sample][unit]
// in LDS, and wave w accumulates rows 32 w .. 32 w + 31 against the 32 columns for every coefficient
// and both parts (64 accumulator registers for two coefficients), so that three workgroups share a
// CU and one's staging overlaps another's products.  The tile after the current one is loaded into
// registers while the products run.  Chunk sums are written in FP32 and added across chunks in FP64.
// coef kinds: 0 -> c = w; 1 -> c = w R; 2 -> c = w u (u double2 [n]);
//             3 -> c = 2 (1 - R) conj(R) / n; 4 -> c = w (R - u[0]) (u pointing at <R>: the centred
//             ratio, whose contraction <O^* (R - <R>)> = <O^* R> - <O^*><R> carries no cancellation of
//             the mean of O)
constexpr int OM_R = 128, OM_C = 32, OM_S = 32;

typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

// the value a binary32 takes after rounding to bfloat16 (nearest, ties to even)
__device__ __forceinline__ float round_to_bf16(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return __uint_as_float(u & 0xFFFF0000u);
}

__device__ __forceinline__ float2 coef_of(int kind, long s, const double* w, double wdef, const float2* R,
                                          const double2* u, double two_over_n) {
    const float ws = w ? (float)w[s] : (float)wdef;
    switch (kind) {
        case 0: return make_float2(ws, 0.f);
        case 1: return cscale(R[s], ws);
        case 2: return make_float2((float)(u[s].x) * ws, (float)(u[s].y) * ws);
        case 4: return cscale(csub(R[s], make_float2((float)u[0].x, (float)u[0].y)), ws);
        default: {
            const float2 r = R[s];
            const float2 d = cmul(make_float2(1.f - r.x, -r.y), cconj(r));
            return cscale(d, (float)two_over_n);
        }
    }
}

// sigma~ rows of the contraction, packed once per call: sites 0..N-1, then 1 (the b row), then zeros up
// to a multiple of 16 sites, so that a thread reads its 16 sites with one aligned 16-byte load.
__global__ void k_pack_sig16(const int8_t* __restrict__ sig, long n, int N, int row, int8_t* __restrict__ out) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * row) return;
    const long s = e / row;
    const int i = (int)(e % row);
    out[e] = i < N ? sig[s * N + i] : (int8_t)(i == N ? 1 : 0);
}

// One sample tile's raw operands in registers: the tile after the current one is loaded while the
// matrix cores work on the current one, so the loads' latency is hidden behind the products.  Thread t
// holds sample t / 8 of the tile with sites 16 (t % 8) .. + 15 of the block and units 4 (t % 8) .. + 3.
template <int NK>
struct OtRaw {
    float sg[16];   // sigma~
    float2 t[4];    // conj(t~)
    float2 cf;      // coefficient of sample t % 32 (t < NK * 32)
};

template <int NK>
__device__ __forceinline__ void ot_load(OtRaw<NK>& r, int tid, int row, int M, int i0, int j0, long sb, long s_end,
                                        const int8_t* __restrict__ sig16, const float2* __restrict__ T, int kind0,
                                        int kind1, const double* __restrict__ w, double wdef,
                                        const float2* __restrict__ R, const double2* __restrict__ u,
                                        double two_over_n, int round_bf16, const double2* __restrict__ shift_b) {
    const long s = sb + (tid >> 3);
    const int g = tid & 7;
    const bool in = s < s_end;
    const int base = i0 + 16 * g;   // a multiple of 16, as is the packed row length
    int4 v = make_int4(0, 0, 0, 0);
    if (in && base < row) v = *reinterpret_cast<const int4*>(sig16 + s * row + base);
    const int word[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int k = 0; k < 16; ++k) r.sg[k] = (float)(int8_t)(word[k >> 2] >> (8 * (k & 3)));
    const float2* trow = T + s * M;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int j = j0 + 4 * g + k;
        float2 t = make_float2(0.f, 0.f);
        if (in && j <= M) t = (j == M) ? make_float2(1.f, 0.f) : trow[j];
        if (shift_b && in && j < M) {
            const double2 c = shift_b[j];
            t = make_float2(t.x - (float)c.x, t.y - (float)c.y);
        }
        if (round_bf16) t = make_float2(round_to_bf16(t.x), round_to_bf16(t.y));
        r.t[k] = cconj(t);
    }
    r.cf = make_float2(0.f, 0.f);
    if (tid < NK * OM_S) {
        const long sc = sb + tid % OM_S;
        if (sc < s_end) r.cf = coef_of(tid / OM_S == 0 ? kind0 : kind1, sc, w, wdef, R, u, two_over_n);
    }
}

// Stage one tile from registers into LDS (two barriers), then issue the loads of the tile after it.
template <int NK>
__device__ __forceinline__ void ot_stage(OtRaw<NK>& raw, float (&sA)[OM_S][OM_R + 4],
                                         float (&sY)[NK][2][OM_S][OM_C], float2 (&sC)[NK][OM_S], int tid, int row,
                                         int M, int i0, int j0, long sb, long s_end, const int8_t* __restrict__ sig16,
                                         const float2* __restrict__ T, int kind0, int kind1,
                                         const double* __restrict__ w, double wdef, const float2* __restrict__ R,
                                         const double2* __restrict__ u, double two_over_n, int round_bf16,
                                         const double2* __restrict__ shift_b) {
    const int ss = tid >> 3, g = tid & 7;
    if (tid < NK * OM_S) sC[tid / OM_S][tid % OM_S] = raw.cf;
#pragma unroll
    for (int k = 0; k < 16; ++k) sA[ss][16 * g + k] = raw.sg[k];
    __syncthreads();
#pragma unroll
    for (int c = 0; c < NK; ++c) {
        const float2 cf = sC[c][ss];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const float2 y = cmul(raw.t[k], cf);
            sY[c][0][ss][4 * g + k] = y.x;
            sY[c][1][ss][4 * g + k] = y.y;
        }
    }
    __syncthreads();
    // the next tile's loads, in flight during the products
    if (sb + OM_S < s_end)
        ot_load<NK>(raw, tid, row, M, i0, j0, sb + OM_S, s_end, sig16, T, kind0, kind1, w, wdef, R, u, two_over_n,
                    round_bf16, shift_b);
}

// One coefficient vector: four waves per SIMD in 128 registers; two: three waves in 168 (no spills in
// either, the matrix-core accumulators among the vector registers).
template <int NK>
__global__ __launch_bounds__(256, NK == 1 ? 4 : 3) void k_ot(int N, int M, int row, const int8_t* __restrict__ sig16,
                                            const float2* __restrict__ T,
                                            long n, long chunk, int n_chunks, int kind0, int kind1,
                                            const double* __restrict__ w, const float2* __restrict__ R,
                                            const double2* __restrict__ u, float* __restrict__ partial,
                                            const double* __restrict__ skip, int round_bf16,
                                            const double2* __restrict__ shift_b) {
    if (skip && *skip != 0.0) return;
    __shared__ __align__(16) float sA[OM_S][OM_R + 4];      // sigma~ [sample][site]
    __shared__ __align__(16) float sY[NK][2][OM_S][OM_C];   // y [c][Re/Im][sample][unit]
    __shared__ float2 sC[NK][OM_S];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int i0 = blockIdx.x * OM_R, j0 = blockIdx.y * OM_C;
    const double wdef = 1.0 / (double)n;
    const double two_over_n = 2.0 / (double)n;
    const int j = j0 + (lane & 31);
    const long plane = (long)(N + 1) * (M + 1);
    // chunks ck = blockIdx.z, blockIdx.z + gridDim.z, ...: each summed in FP32 on its own
    for (int ck = blockIdx.z; ck < n_chunks; ck += gridDim.z) {
        const long s_begin = (long)ck * chunk;
        const long s_end = min(n, s_begin + chunk);
        OtRaw<NK> raw;
        ot_load<NK>(raw, tid, row, M, i0, j0, s_begin, s_end, sig16, T, kind0, kind1, w, wdef, R, u, two_over_n,
                    round_bf16, shift_b);
        if (i0 + 32 * wv > N) {
            // no extended site in this wave's rows: it only helps to stage the tiles
            for (long sb = s_begin; sb < s_end; sb += OM_S) {
                ot_stage<NK>(raw, sA, sY, sC, tid, row, M, i0, j0, sb, s_end, sig16, T, kind0, kind1, w, wdef, R, u,
                             two_over_n, round_bf16, shift_b);
                __syncthreads();
            }
            continue;
        }
        f32x16 acc[NK][2];
#pragma unroll
        for (int c = 0; c < NK; ++c)
#pragma unroll
            for (int ri = 0; ri < 2; ++ri)
#pragma unroll
                for (int v = 0; v < 16; ++v) acc[c][ri][v] = 0.f;
        for (long sb = s_begin; sb < s_end; sb += OM_S) {
            ot_stage<NK>(raw, sA, sY, sC, tid, row, M, i0, j0, sb, s_end, sig16, T, kind0, kind1, w, wdef, R, u,
                         two_over_n, round_bf16, shift_b);
            // lane l supplies row l % 32 (A) and column l % 32 (B) at sample 2 ks + l / 32; rows past N are zeros
#pragma unroll 4
            for (int ks = 0; ks < OM_S / 2; ++ks) {
                const int kk = 2 * ks + (lane >> 5);
                const float a = sA[kk][32 * wv + (lane & 31)];
#pragma unroll
                for (int c = 0; c < NK; ++c)
#pragma unroll
                    for (int ri = 0; ri < 2; ++ri)
                        acc[c][ri] =
                            __builtin_amdgcn_mfma_f32_32x32x2f32(a, sY[c][ri][kk][lane & 31], acc[c][ri], 0, 0, 0);
            }
            __syncthreads();
        }
        // accumulator element v of lane l: row 8(v/4) + 4(l/32) + v%4 of the fragment, column l % 32;
        // the chunk's FP32 sums go to planes [chunk][c][Re/Im] straight from the accumulators
        if (j <= M) {
#pragma unroll
            for (int c = 0; c < NK; ++c)
#pragma unroll
                for (int ri = 0; ri < 2; ++ri) {
                    float* out = partial + (((long)ck * NK + c) * 2 + ri) * plane + j;
#pragma unroll
                    for (int v = 0; v < 16; ++v) {
                        const int i = i0 + 32 * wv + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
                        if (i <= N) out[(long)i * (M + 1)] = acc[c][ri][v];
                    }
                }
        }
    }
}

// out[c][P-index] = sum over chunks of the FP32 chunk sums (in FP64), with optional conjugation.  With
// shift_b: the chunks summed conj(T - c_j) for the units j < M, and conj(c_j) times the same coefficient
// vector's sum over sigma~_i (its column j = M) is added back here; for coefficient vector 0 (the weights)
// that sum is exactly 1 on the b row.
__global__ void k_ot_reduce(int N, int M, const float* __restrict__ partial, int n_chunks, int nk, int conj0,
                            double2* __restrict__ out0, double2* __restrict__ out1, const double* __restrict__ skip,
                            const double2* __restrict__ shift_b) {
    if (skip && *skip != 0.0) return;
    const long plane = (long)(N + 1) * (M + 1);
    const long o = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= plane) return;
    const int i = (int)(o / (M + 1)), j = (int)(o % (M + 1));
    if (i == N && j == M) return;
    const long k = ij_to_p(i, j, N, M);
    for (int c = 0; c < nk; ++c) {
        double2 acc = make_double2(0.0, 0.0);
        for (int b = 0; b < n_chunks; ++b) {
            const float* pc = partial + ((long)b * nk + c) * 2 * plane;
            acc.x += (double)pc[o];
            acc.y += (double)pc[plane + o];
        }
        if (shift_b && j < M) {
            double2 y = make_double2(1.0, 0.0);
            if (i < N || c > 0) {
                const long oy = (long)i * (M + 1) + M;
                y = make_double2(0.0, 0.0);
                for (int b = 0; b < n_chunks; ++b) {
                    const float* pc = partial + ((long)b * nk + c) * 2 * plane;
                    y.x += (double)pc[oy];
                    y.y += (double)pc[plane + oy];
                }
            }
            const double2 cj = make_double2((double)(float)shift_b[j].x, (double)(float)shift_b[j].y);
            acc = zadd(acc, zconjmul(cj, y));
        }
        if (c == 0 && conj0) acc.y = -acc.y;
        (c == 0 ? out0 : out1)[k] = acc;
    }
}

// Sample chunks of at least n/256 and at least 256 samples (a multiple of the 32-sample tile), at most
// 256 of them, which the plan's reduction buffer holds (it has room for min(ceil(n / 256), 257)
// chunks); each chunk is summed in FP32 on its own, as many samples as on the vector units before.
// The grid holds as many workgroups as the device keeps resident at once (the kernel's occupancy
// times the CUs, so that no second, nearly empty round follows); each loops over its chunks.
struct OtPlan { long chunk; int n_chunks; int grid_z; };
template <int NK>
static int ot_resident_per_cu() {
    static int cached = 0;
    if (!cached) {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_ot<NK>, 256, 0) != hipSuccess || nb < 1) nb = 1;
        cached = nb;
    }
    return cached;
}
static void ot_chunking(long n, long& chunk, int& n_chunks) {
    chunk = (n + 255) / 256;
    chunk = ((chunk + OM_S - 1) / OM_S) * OM_S;
    if (chunk < 256) chunk = 256;
    n_chunks = (int)((n + chunk - 1) / chunk);
}
static OtPlan ot_plan(int N, int M, long n, int nk, int n_cu) {
    long chunk;
    int n_chunks;
    ot_chunking(n, chunk, n_chunks);
    const long tiles = (long)((N + 1 + OM_R - 1) / OM_R) * ((M + 1 + OM_C - 1) / OM_C);
    const long slots = (long)n_cu * (nk == 2 ? ot_resident_per_cu<2>() : ot_resident_per_cu<1>());
    long z = slots / tiles;
    if (z < 1) z = 1;
    if (z > n_chunks) z = n_chunks;
    // the same number of chunks for every workgroup where possible
    z = (n_chunks + ((n_chunks + z - 1) / z) - 1) / ((n_chunks + z - 1) / z);
    return {chunk, n_chunks, (int)z};
}

// sig16: the packed sigma~ rows (k_pack_sig16) of the n samples; partial: scratch of at least
// 2 nk (N + 1)(M + 1) floats per chunk
static hipError_t run_ot(int N, int M, const int8_t* sig16, const float2* T, long n, int kind0, int kind1, int nk,
                         const double* w, const float2* R, const double2* u, void* partial_buf, int conj0,
                         double2* out0, double2* out1, hipStream_t stream, const double* skip, Profiler* prof,
                         int n_cu, int round_bf16 = 0, const double2* shift_b = nullptr) {
    const OtPlan op = ot_plan(N, M, n, nk, n_cu);
    const int row = sig16_row(N);
    float* partial = static_cast<float*>(partial_buf);
    dim3 grid((N + 1 + OM_R - 1) / OM_R, (M + 1 + OM_C - 1) / OM_C, op.grid_z);
    if (prof) prof->begin(PROF_OT, stream);
    if (nk == 2)
        hipLaunchKernelGGL(k_ot<2>, grid, dim3(256), 0, stream, N, M, row, sig16, T, n, op.chunk, op.n_chunks, kind0,
                           kind1, w, R, u, partial, skip, round_bf16, shift_b);
    else
        hipLaunchKernelGGL(k_ot<1>, grid, dim3(256), 0, stream, N, M, row, sig16, T, n, op.chunk, op.n_chunks, kind0,
                           kind1, w, R, u, partial, skip, round_bf16, shift_b);
    if (prof) prof->end(stream);
    const long plane = (long)(N + 1) * (M + 1);
    hipLaunchKernelGGL(k_ot_reduce, dim3((unsigned)((plane + 255) / 256)), dim3(256), 0, stream, N, M, partial,
                       op.n_chunks, nk, conj0, out0, out1, skip, shift_b);
    return hipGetLastError();
}

static void pack_sig16(const int8_t* sig, long n, int N, int8_t* out, hipStream_t stream) {
    const long cnt = n * (long)sig16_row(N);
    hipLaunchKernelGGL(k_pack_sig16, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, stream, sig, n, N,
                       sig16_row(N), out);
}

// ORc = <O^* (R - <R>)> = <O^* R> - <O^*><R>  (R = E_loc in energy mode):
// fit mode (0):    F_k = coef [<O_k^* R>/<R> - <O_k^*>] = coef ORc_k / <R>;
// energy mode (1): F_k = coef [<O_k^* E> - <O_k^*><E>] = coef ORc_k   (coef = -lr).
// Om holds conj(<O>) on entry and <O> on exit.
__global__ void k_make_f(long P, int mode, double2* __restrict__ Om, const double2* __restrict__ ORm,
                         const double* __restrict__ sc, double2* __restrict__ F) {
    const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= P) return;
    const double2 rm = make_double2(sc[SC_RM_RE], sc[SC_RM_IM]);
    const double coef = sc[SC_COEF];
    const double2 omc = Om[k];
    const double2 d = mode == 1 ? ORm[k] : zdiv(ORm[k], rm);
    F[k] = make_double2(coef * d.x, coef * d.y);
    Om[k] = make_double2(omc.x, -omc.y);
}

// F alone from ORc (as k_make_f, the means left as they are)
__global__ void k_f_of(long P, int mode, const double2* __restrict__ ORm, const double* __restrict__ sc,
                       double2* __restrict__ F) {
    const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= P) return;
    const double2 rm = make_double2(sc[SC_RM_RE], sc[SC_RM_IM]);
    const double coef = sc[SC_COEF];
    const double2 d = mode == 1 ? ORm[k] : zdiv(ORm[k], rm);
    F[k] = make_double2(coef * d.x, coef * d.y);
}

// ------------------------------------------------------------------ weighted P-vector contractions in double
// With sample weights (exact enumeration: every configuration once, weighted by |psi|^2 / Z) the weights span
// many orders of magnitude and the configurations next to nodes of the state carry O_k of the same size
// inverted, so the sums over samples run in double here: Om_k = sum_s w_s conj(O_sk) and
// ORc_k = sum_s w_s conj(O_sk) (R_s - <R>).  One thread per parameter; threads of one site row read
// consecutive hidden units of T.
__global__ __launch_bounds__(256) void k_ot64(int N, int M, long P, const int8_t* __restrict__ sig,
                                              const float2* __restrict__ T, const double* __restrict__ w,
                                              const float2* __restrict__ R, long n, const double* __restrict__ sc,
                                              double2* __restrict__ Om, double2* __restrict__ ORc) {
    const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= P) return;
    int i, j;
    p_to_ij(k, N, M, i, j);
    const double rx = sc[SC_RM_RE], ry = sc[SC_RM_IM];
    double ox = 0, oy = 0, qx = 0, qy = 0;
    for (long s = 0; s < n; ++s) {
        const double ws = w[s];
        const double sv = (i == N) ? 1.0 : (double)sig[s * N + i];
        double tx = 1.0, ty = 0.0;
        if (j < M) { const float2 t = T[s * M + j]; tx = t.x; ty = t.y; }
        const double cx = ws * sv * tx, cy = -ws * sv * ty;          // w conj(O)
        const double dx = (double)R[s].x - rx, dy = (double)R[s].y - ry;
        ox += cx; oy += cy;
        qx += cx * dx - cy * dy; qy += cx * dy + cy * dx;
    }
    Om[k] = make_double2(ox, oy);
    ORc[k] = make_double2(qx, qy);
}

// ------------------------------------------------------------------ dense S (FP32, VALU)
// Upper-triangle tiles (I <= J) of 64 x 64, mirrored into the lower triangle so that S is stored in full:
//   S[k][k'] = sum_s w conj(O_sk - m_k) (O_sk' - m_k') + (1 - sum_s w) conj(m_k) m_k',  m = <O>,
// which is <O^* O> - <O>^* <O> (Sec. III) with the operands centred before the sums: where |<O_k>|^2 is
// large against the variance (tanh theta near +-1), raw sums less the product of the means would lose that
// ratio's digits.  Binary32 operands, products and sums in double (the weighted sums serve exact enumeration
// with a dense solve, where a few configurations next to nodes of the state can make |S| large against the
// diagonal shift); S is written in binary32 and, for the Cholesky solve, also in double (S64).
constexpr int SB_T = 64, SB_K = 16;

__global__ __launch_bounds__(256) void k_sbuild(int N, int M, long P, const int8_t* __restrict__ sig,
                                                const float2* __restrict__ T, const double* __restrict__ w, long n,
                                                const double2* __restrict__ Om, float2* __restrict__ S, int ntile,
                                                const double* __restrict__ sc, double2* __restrict__ S64) {
    __shared__ float2 sa[SB_K][SB_T];
    __shared__ float2 sb[SB_K][SB_T];
    // map blockIdx.x -> (I, J), I <= J
    long rem = blockIdx.x;
    int I = 0;
    while (rem >= ntile - I) { rem -= ntile - I; ++I; }
    const int J = I + (int)rem;
    const int tid = threadIdx.x, ty = tid >> 4, tx = tid & 15;
    const long kA0 = (long)I * SB_T, kB0 = (long)J * SB_T;
    // columns loaded by this thread: column c = tid & 63, rows ss = tid >> 6 (+4 steps)
    const int lc = tid & 63;
    int ia, ja, ib, jb;
    const bool va = kA0 + lc < P, vb = kB0 + lc < P;
    p_to_ij(va ? kA0 + lc : 0, N, M, ia, ja);
    p_to_ij(vb ? kB0 + lc : 0, N, M, ib, jb);
    const double2 mA = va ? Om[kA0 + lc] : make_double2(0.0, 0.0), mB = vb ? Om[kB0 + lc] : make_double2(0.0, 0.0);
    const float2 mAf = make_float2((float)mA.x, (float)mA.y), mBf = make_float2((float)mB.x, (float)mB.y);
    const double wdef = 1.0 / (double)n;
    double2 acc[4][4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[r][c] = make_double2(0.0, 0.0);

    for (long s0 = 0; s0 < n; s0 += SB_K) {
#pragma unroll
        for (int st = 0; st < SB_K / 4; ++st) {
            const int ss = (tid >> 6) + 4 * st;
            const long s = s0 + ss;
            float2 oa = make_float2(0.f, 0.f), ob = make_float2(0.f, 0.f);
            if (s < n) {
                const float ws = w ? (float)w[s] : (float)wdef;
                if (va) {
                    const float sv = (ia == N) ? 1.f : (float)sig[s * N + ia];
                    const float2 tv = (ja == M) ? make_float2(1.f, 0.f) : T[s * M + ja];
                    oa = cscale(cconj(csub(cscale(tv, sv), mAf)), ws);
                }
                if (vb) {
                    const float sv = (ib == N) ? 1.f : (float)sig[s * N + ib];
                    const float2 tv = (jb == M) ? make_float2(1.f, 0.f) : T[s * M + jb];
                    ob = csub(cscale(tv, sv), mBf);
                }
            }
            sa[ss][lc] = oa;
            sb[ss][lc] = ob;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < SB_K; ++kk) {
            float2 av[4], bv[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) av[r] = sa[kk][ty + 16 * r];
#pragma unroll
            for (int c = 0; c < 4; ++c) bv[c] = sb[kk][tx + 16 * c];
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const double ax = av[r].x, ay = av[r].y, bx = bv[c].x, by = bv[c].y;
                    acc[r][c].x = fma(ax, bx, fma(-ay, by, acc[r][c].x));
                    acc[r][c].y = fma(ax, by, fma(ay, bx, acc[r][c].y));
                }
        }
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const long k = kA0 + ty + 16 * r;
        if (k >= P) continue;
        const double2 omk = Om[k];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const long kp = kB0 + tx + 16 * c;
            if (kp >= P) continue;
            const double2 omkp = Om[kp];
            const double2 mm = zconjmul(omk, omkp);
            const double rest = 1.0 - sc[SC_WSUM];
            const double2 d = make_double2(acc[r][c].x + rest * mm.x, acc[r][c].y + rest * mm.y);
            const float2 v = make_float2((float)d.x, (float)d.y);
            S[k * P + kp] = v;
            if (I != J) S[kp * P + k] = cconj(v);
            if (S64) {
                S64[k * P + kp] = d;
                if (I != J) S64[kp * P + k] = make_double2(d.x, -d.y);
            }
        }
    }
}

// ------------------------------------------------------------------ dense Hermitian product
// y = (S + eps I) x with S complex64 [P][P] read from its lower triangle only, x and y complex128.
// Tile (I, J), J <= I, of HV_T x HV_T entries gives S_IJ x_J to the rows of I and, for J < I, also
// S_IJ^H x_I to the rows of J (the upper triangle is never read, halving the bytes of a product).
// Each partial vector has its own slot, part[A][B] = the share of tile pair {A, B} in y_A, and a
// second pass adds the nT slots of every row in the same order (deterministic).
constexpr int HV_T = kHemvTile;

// PAIR (P even, so every row and tile starts on 16 bytes): a lane reads two adjacent columns per load,
// columns 2 c0 + 32 j' + {0, 1}; otherwise one column, c0 + 16 j.
template <bool PAIR>
__global__ __launch_bounds__(256) void k_hemv_tiles(long P, int nT, const float2* __restrict__ S,
                                                    const double2* __restrict__ x, double2* __restrict__ part,
                                                    const double* __restrict__ sc) {
    if (sc[SC_DONE] != 0.0) return;
    // lower-triangle tile (I, J) of this workgroup: t = I (I + 1) / 2 + J
    const long t = blockIdx.x;
    int I = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while ((long)I * (I + 1) / 2 > t) --I;
    while ((long)(I + 1) * (I + 2) / 2 <= t) ++I;
    const int J = (int)(t - (long)I * (I + 1) / 2);
    __shared__ double2 xI[HV_T], xJ[HV_T];
    __shared__ double2 cred[4][HV_T];
    const int tid = threadIdx.x;
    const long i0 = (long)I * HV_T, j0 = (long)J * HV_T;
    xI[tid] = i0 + tid < P ? x[i0 + tid] : make_double2(0.0, 0.0);
    xJ[tid] = j0 + tid < P ? x[j0 + tid] : make_double2(0.0, 0.0);
    __syncthreads();
    // a 16-lane group takes one row at a time, so that every load instruction of a group covers
    // 128 (256 with PAIR) contiguous bytes of the row
    const int lane = tid & 63, w = tid >> 6, g = lane >> 4, c0 = lane & 15;
    const int nrows = (int)(P - i0 < HV_T ? P - i0 : HV_T);
    const int ncols = (int)(P - j0 < HV_T ? P - j0 : HV_T);
    double cx[16], cy[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) { cx[j] = 0.0; cy[j] = 0.0; }
    for (int rr = 4 * w + g; rr < nrows; rr += 16) {
        const float2* Sr = S + (i0 + rr) * P + j0;
        const double2 xi = xI[rr];
        double rx = 0.0, ry = 0.0;
#pragma unroll
        for (int jp = 0; jp < (PAIR ? 8 : 16); ++jp) {
            float2 sv2[2];
            if constexpr (PAIR) {
                const int c = 2 * c0 + 32 * jp;
                // columns past P: read columns 0, 1 instead; x_J is zero there and the column share is unused
                const float4 v4 = *reinterpret_cast<const float4*>(Sr + (c < ncols ? c : 0));
                sv2[0] = make_float2(v4.x, v4.y);
                sv2[1] = make_float2(v4.z, v4.w);
            } else {
                const int c = c0 + 16 * jp;
                sv2[0] = Sr[c < ncols ? c : 0];
            }
#pragma unroll
            for (int h = 0; h < (PAIR ? 2 : 1); ++h) {
                const int j = PAIR ? 2 * jp + h : jp;
                const int c = PAIR ? 2 * c0 + 32 * jp + h : c0 + 16 * jp;
                const double sx = sv2[h].x, sy = sv2[h].y;
                const double2 xj = xJ[c];
                rx += sx * xj.x - sy * xj.y;
                ry += sx * xj.y + sy * xj.x;
                cx[j] += sx * xi.x + sy * xi.y;            // conj(S_rc) x_r
                cy[j] += sx * xi.y - sy * xi.x;
            }
        }
#pragma unroll
        for (int o = 8; o >= 1; o >>= 1) {
            rx += __shfl_xor(rx, o, 16);
            ry += __shfl_xor(ry, o, 16);
        }
        if (c0 == 0) part[((long)I * nT + J) * HV_T + rr] = make_double2(rx, ry);
    }
    if (J == I) return;                              // the diagonal tile was read in full
    // column shares: add the 4 row groups of the wave, then the 4 waves in order
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        cx[j] += __shfl_xor(cx[j], 16);
        cy[j] += __shfl_xor(cy[j], 16);
        cx[j] += __shfl_xor(cx[j], 32);
        cy[j] += __shfl_xor(cy[j], 32);
    }
    if (g == 0)
#pragma unroll
        for (int j = 0; j < 16; ++j) cred[w][PAIR ? 2 * c0 + 32 * (j >> 1) + (j & 1) : c0 + 16 * j] = make_double2(cx[j], cy[j]);
    __syncthreads();
    const double2 a = cred[0][tid], b = cred[1][tid], c = cred[2][tid], d = cred[3][tid];
    part[((long)J * nT + I) * HV_T + tid] = make_double2(((a.x + b.x) + c.x) + d.x, ((a.y + b.y) + c.y) + d.y);
}

// y_k = sum_B part[k / HV_T][B][k % HV_T] + eps x_k; 64 rows per workgroup, its 4 waves add a quarter
// of the slots each, combined in wave order
__global__ __launch_bounds__(256) void k_hemv_reduce(long P, int nT, const double2* __restrict__ part,
                                                     const double2* __restrict__ x, double eps,
                                                     double2* __restrict__ y, const double* __restrict__ sc) {
    if (sc[SC_DONE] != 0.0) return;
    __shared__ double2 q[4][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const long k = (long)blockIdx.x * 64 + lane;
    double sx = 0.0, sy = 0.0;
    if (k < P) {
        const long I = k / HV_T, r = k % HV_T;
        const double2* pr = part + I * nT * HV_T + r;
        const int per = (nT + 3) / 4;
        const int b0 = w * per, b1 = b0 + per < nT ? b0 + per : nT;
#pragma unroll 8
        for (int B = b0; B < b1; ++B) {
            const double2 v = pr[(long)B * HV_T];
            sx += v.x;
            sy += v.y;
        }
    }
    q[w][lane] = make_double2(sx, sy);
    __syncthreads();
    if (w == 0 && k < P) {
        const double2 a = q[0][lane], b = q[1][lane], c = q[2][lane], d = q[3][lane];
        y[k] = make_double2((((a.x + b.x) + c.x) + d.x) + eps * x[k].x, (((a.y + b.y) + c.y) + d.y) + eps * x[k].y);
    }
}

// ------------------------------------------------------------------ matrix-free S v
// u_s = sum_j T~_sj G_sj + sum_i sigma_si v_a_i with G = theta-GEMM(b = v_b, W = v_W)
__global__ __launch_bounds__(256) void k_pack_v(int N, int M, const double2* __restrict__ v, float2* __restrict__ vb,
                                                float2* __restrict__ vW, const double* __restrict__ sc) {
    if (sc[SC_DONE] != 0.0) return;
    const long P = (long)N + M + (long)N * M;
    const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < N || k >= P) return;
    const float2 f = make_float2((float)v[k].x, (float)v[k].y);
    if (k < N + M) vb[k - N] = f; else vW[k - N - M] = f;
}


// u <- u - <O>.v (scalar), so that the contraction gives <O^*(O v)> - <O>^* <O>.v with <O^*> folded.
__global__ __launch_bounds__(256) void k_dot_ov(long P, const double2* __restrict__ Om, const double2* __restrict__ v,
                                                double2* __restrict__ red, const double* __restrict__ sc) {
    if (sc[SC_DONE] != 0.0) return;
    __shared__ double sh[2][4];
    double ax = 0, ay = 0;
    for (long k = (long)blockIdx.x * 256 + threadIdx.x; k < P; k += (long)gridDim.x * 256) {
        const double2 t = zmul(Om[k], v[k]);
        ax += t.x; ay += t.y;
    }
    ax = wave_sum(ax); ay = wave_sum(ay);
    if ((threadIdx.x & 63) == 0) { sh[0][threadIdx.x >> 6] = ax; sh[1][threadIdx.x >> 6] = ay; }
    __syncthreads();
    if (threadIdx.x == 0) red[blockIdx.x] = make_double2(sh[0][0] + sh[0][1] + sh[0][2] + sh[0][3],
                                                         sh[1][0] + sh[1][1] + sh[1][2] + sh[1][3]);
}

__global__ __launch_bounds__(256) void k_sub_mean(long n, double2* __restrict__ u, const double2* __restrict__ red,
                                                  int n_red, const double* __restrict__ sc) {
    if (sc[SC_DONE] != 0.0) return;
    double2 m = make_double2(0.0, 0.0);
    for (int b = 0; b < n_red; ++b) m = zadd(m, red[b]);
    const long s = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s < n) u[s] = make_double2(u[s].x - m.x, u[s].y - m.y);
}

__global__ void k_add_shift(long P, const double2* __restrict__ x, double eps, double2* __restrict__ y,
                            const double* __restrict__ sc) {
    if (sc[SC_DONE] != 0.0) return;
    const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < P) y[k] = make_double2(y[k].x + eps * x[k].x, y[k].y + eps * x[k].y);
}

// ------------------------------------------------------------------ CG helpers (double)
// red[blk] = sum conj(a) b over the block's range
__global__ __launch_bounds__(256) void k_zdot(long P, const double2* __restrict__ a, const double2* __restrict__ b,
                                              double2* __restrict__ red, const double* __restrict__ sc, int check) {
    if (check && sc[SC_DONE] != 0.0) return;
    __shared__ double sh[2][4];
    double ax = 0, ay = 0;
    for (long k = (long)blockIdx.x * 256 + threadIdx.x; k < P; k += (long)gridDim.x * 256) {
        const double2 t = zconjmul(a[k], b[k]);
        ax += t.x; ay += t.y;
    }
    ax = wave_sum(ax); ay = wave_sum(ay);
    if ((threadIdx.x & 63) == 0) { sh[0][threadIdx.x >> 6] = ax; sh[1][threadIdx.x >> 6] = ay; }
    __syncthreads();
    if (threadIdx.x == 0) red[blockIdx.x] = make_double2(sh[0][0] + sh[0][1] + sh[0][2] + sh[0][3],
                                                         sh[1][0] + sh[1][1] + sh[1][2] + sh[1][3]);
}

// slot <- Re sum(red)
__global__ void k_sum_to(const double2* __restrict__ red, int n_red, double* __restrict__ sc, int slot, int check) {
    if (check && sc[SC_DONE] != 0.0) return;
    if (threadIdx.x != 0) return;
    double a = 0;
    for (int b = 0; b < n_red; ++b) a += red[b].x;
    sc[slot] = a;
}

// real part of red[0] + ... + red[n-1] in one fixed order, the same in every block (256 threads)
__device__ __forceinline__ double block_sum_re(const double2* __restrict__ red, int n, double* sh) {
    double a = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) a += red[i].x;
    sh[threadIdx.x] = a;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    const double t = sh[0];
    __syncthreads();
    return t;
}

// x += alpha p, r -= alpha Ap with alpha = rr / pAp (pAp from the 64 partials of k_zdot, rr in slot
// `slot`); each block leaves its part of the new r^H r in red_rr[block]
__global__ __launch_bounds__(256) void k_cg_xr(long P, double2* __restrict__ x, double2* __restrict__ r,
                                               const double2* __restrict__ p, const double2* __restrict__ Ap,
                                               const double2* __restrict__ red_pap, double2* __restrict__ red_rr,
                                               double* __restrict__ sc, int slot) {
    __shared__ double sh[256];
    if (sc[SC_DONE] != 0.0) return;              // set only by k_cg_check_p: fixed during this launch
    const double pap = block_sum_re(red_pap, 64, sh);
    const double alpha = sc[slot] / pap;
    const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
    double rr = 0.0;
    if (k < P) {
        x[k] = make_double2(x[k].x + alpha * p[k].x, x[k].y + alpha * p[k].y);
        const double2 rk = make_double2(r[k].x - alpha * Ap[k].x, r[k].y - alpha * Ap[k].y);
        r[k] = rk;
        rr = rk.x * rk.x + rk.y * rk.y;
    }
    sh[threadIdx.x] = rr;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        red_rr[blockIdx.x] = make_double2(sh[0], 0.0);
        if (blockIdx.x == 0) sc[SC_PAP] = pap;
    }
}

// Convergence test of iteration `it` and the direction update p = r + beta p.  Every block adds the
// r^H r partials in the same order and takes the same decision; block 0 records it: the new r^H r goes
// to the other slot than the one read, so no block reads a slot written in this launch.
__global__ __launch_bounds__(256) void k_cg_check_p(long P, double2* __restrict__ p, const double2* __restrict__ r,
                                                    const double2* __restrict__ red_rr, int n_red,
                                                    double* __restrict__ sc, double tol, int maxit, int it, int slot) {
    __shared__ double sh[256];
    __shared__ int s_done;
    if (threadIdx.x == 0) s_done = sc[SC_DONE] != 0.0;   // block 0 may set it during this launch
    __syncthreads();
    if (s_done) return;
    const double rn = block_sum_re(red_rr, n_red, sh);
    const bool bad = !isfinite(rn) || !(sc[SC_PAP] > 0.0);
    const bool conv = !bad && sqrt(rn) <= tol * sqrt(sc[SC_FF]);
    const bool last = it + 1 >= maxit;
    const int next = slot == SC_RR ? SC_RR1 : SC_RR;
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    if (bad || conv || last) {
        if (lead) {
            int fl = (int)sc[SC_FLAGS];
            if (bad) fl |= CRBM_FLAG_NONFINITE;
            else if (!conv) fl |= CRBM_FLAG_NOT_CONVERGED;
            sc[SC_FLAGS] = (double)fl;
            sc[SC_ITERS] = (double)(it + 1);
            sc[next] = rn;
            sc[SC_DONE] = 1.0;
        }
        return;
    }
    const double beta = rn / sc[slot];
    const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < P) p[k] = make_double2(r[k].x + beta * p[k].x, r[k].y + beta * p[k].y);
    if (lead) {
        sc[next] = rn;
        sc[SC_ITERS] = (double)(it + 1);
    }
}

__global__ __launch_bounds__(256) void k_cg_init(long P, const double2* __restrict__ F, double2* __restrict__ x,
                                                 double2* __restrict__ r, double2* __restrict__ p) {
    const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= P) return;
    x[k] = make_double2(0.0, 0.0);
    r[k] = F[k];
    p[k] = F[k];
}

__global__ void k_cg_start(double* __restrict__ sc) {
    if (threadIdx.x != 0) return;
    sc[SC_RR] = sc[SC_FF];
    sc[SC_DONE] = (sc[SC_FF] == 0.0 || (int)sc[SC_FLAGS] != 0) ? 1.0 : 0.0;
    sc[SC_ITERS] = 0.0;
}

// r = F - Ap (true residual), used once after the iterations
__global__ __launch_bounds__(256) void k_resid(long P, const double2* __restrict__ F, const double2* __restrict__ Ax,
                                               double2* __restrict__ r) {
    const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < P) r[k] = make_double2(F[k].x - Ax[k].x, F[k].y - Ax[k].y);
}

__global__ void k_undone(double* __restrict__ sc) { if (threadIdx.x == 0) sc[SC_DONE] = 0.0; }

// a, b, W += dalpha  (skipped when the step was flagged non-finite)
__global__ __launch_bounds__(256) void k_update(int N, int M, float2* __restrict__ a, float2* __restrict__ b,
                                                float2* __restrict__ W, const double2* __restrict__ x,
                                                const double* __restrict__ sc) {
    if (((int)sc[SC_FLAGS] & (CRBM_FLAG_NONFINITE | CRBM_FLAG_CHOLESKY_FAIL)) != 0) return;
    const long P = (long)N + M + (long)N * M;
    const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= P) return;
    float2* dst = (k < N) ? &a[k] : (k < N + M) ? &b[k - N] : &W[k - N - M];
    *dst = make_float2(dst->x + (float)x[k].x, dst->y + (float)x[k].y);
}

__global__ void k_stats(const double* __restrict__ sc, double* __restrict__ out) {
    if (threadIdx.x != 0) return;
    out[0] = sc[SC_GAMMA];
    out[1] = sc[SC_RM_RE];
    out[2] = sc[SC_RM_IM];
    out[3] = sqrt(sc[SC_FF]);
    out[4] = sc[SC_FF] > 0.0 ? sqrt(sc[SC_RESID] / sc[SC_FF]) : 0.0;
    out[5] = sc[SC_ITERS];
    out[6] = sc[SC_FLAGS];
    out[7] = sqrt(sc[SC_XX]);
}

// ------------------------------------------------------------------ driver
static inline unsigned nblk(long n, int t = 256) { return (unsigned)((n + t - 1) / t); }

hipError_t launch_cholesky_solve(long P, const float2* S, double eps, const double2* F, double2* A64, double2* x,
                                 double* sc, bool a64_holds_s, hipStream_t stream);

static hipError_t apply_op(const SrArgs& A, const SrWork& W, const double2* v, double2* y, hipStream_t stream) {
    const long P = A.P;
    if (A.solver == CRBM_SOLVER_CG_MATFREE) {
        // V = (v_b, v_W) in float for the theta product (b = v_b, W = v_W)
        float2* vb = W.vstage;
        float2* vW = vb + A.M;
        hipLaunchKernelGGL(k_pack_v, dim3(nblk(P)), dim3(256), 0, stream, A.N, A.M, v, vb, vW, W.scal);
        // u = O v per sample, the theta product of V fused with the sum over T (partials in the G scratch)
        hipError_t e = launch_theta_ov(A.samples, A.n, A.N, A.M, vb, vW, v, A.T, W.wplanes,
                                       reinterpret_cast<double2*>(W.G), W.u, stream, W.scal + SC_DONE);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_dot_ov, dim3(64), dim3(256), 0, stream, P, W.Om, v, W.red, W.scal);
        hipLaunchKernelGGL(k_sub_mean, dim3(nblk(A.n)), dim3(256), 0, stream, A.n, W.u, W.red, 64, W.scal);
        e = run_ot(A.N, A.M, W.sig16, A.T, A.n, 2, 0, 1, A.weights, A.R, W.u, W.red + 64, 0, y, nullptr, stream,
                   W.scal + SC_DONE, nullptr, W.n_cu);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_add_shift, dim3(nblk(P)), dim3(256), 0, stream, P, v, A.eps, y, W.scal);
    } else {
        const int nT = hemv_tiles(P);
        const dim3 grid((unsigned)((long)nT * (nT + 1) / 2));
        if (P % 2 == 0)
            hipLaunchKernelGGL(k_hemv_tiles<true>, grid, dim3(256), 0, stream, P, nT, W.S, v, W.hv_part, W.scal);
        else
            hipLaunchKernelGGL(k_hemv_tiles<false>, grid, dim3(256), 0, stream, P, nT, W.S, v, W.hv_part, W.scal);
        hipLaunchKernelGGL(k_hemv_reduce, dim3(nblk(P, 64)), dim3(256), 0, stream, P, nT, W.hv_part, v, A.eps, y,
                           W.scal);
    }
    return hipGetLastError();
}

hipError_t launch_sr_step(const SrArgs& A, const SrWork& W, hipStream_t stream) {
    const long P = A.P;
    hipError_t e;
    // scalars gamma, beta, gamma cot gamma
    const int nb_r = 256;
    hipLaunchKernelGGL(k_r_moments, dim3(nb_r), dim3(256), 0, stream, A.R, A.weights, A.n, W.red);
    hipLaunchKernelGGL(k_r_final, dim3(1), dim3(64), 0, stream, W.red, nb_r, A.dgamma, A.mode, W.scal);
    // conj(<O>) and <O^* (R - <R>)>: FP32 chunk sums on the matrix cores, or in double with sample weights
    pack_sig16(A.samples, A.n, A.N, W.sig16, stream);
    if (A.weights) {
        W.prof->begin(PROF_OT, stream);
        hipLaunchKernelGGL(k_ot64, dim3(nblk(P)), dim3(256), 0, stream, A.N, A.M, P, A.samples, A.T, A.weights, A.R,
                           A.n, W.scal, W.Om, W.ORm);
        W.prof->end(stream);
        e = hipGetLastError();
    } else {
        e = run_ot(A.N, A.M, W.sig16, A.T, A.n, 0, 4, 2, A.weights, A.R,
                   reinterpret_cast<const double2*>(W.scal + SC_RM_RE), W.red, 0, W.Om, W.ORm, stream, nullptr, W.prof,
                   W.n_cu);
    }
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_make_f, dim3(nblk(P)), dim3(256), 0, stream, P, A.mode, W.Om, W.ORm, W.scal, W.F);
    hipLaunchKernelGGL(k_zdot, dim3(64), dim3(256), 0, stream, P, W.F, W.F, W.red, W.scal, 0);
    hipLaunchKernelGGL(k_sum_to, dim3(1), dim3(64), 0, stream, W.red, 64, W.scal, (int)SC_FF, 0);

    if (A.solver != CRBM_SOLVER_CG_MATFREE) {
        if (A.weights == nullptr) {
            // The contraction sees T' = T - c (c = <T> in binary32; rounded to BF16 with BF16 operands).
            // The subtracted means are those of the same operands, T' + c, summed as T' in the chunks
            // with c <sigma~> added in double: S stays the centred Gram matrix of one set of vectors
            // (positive semi-definite) and no sum carries |c|^2 against the spread of T.
            if (A.prec == CRBM_PREC_BF16) {
                // F from the same rounded operands: the step then solves the ridge problem of one set of
                // vectors, min |O~ x - D|^2 + eps |x|^2.  With F from the unrounded O, the part of
                // <O^* D> outside the span of the rounded O~ would be divided by eps.
                e = run_ot(A.N, A.M, W.sig16, A.T, A.n, 0, 4, 2, nullptr, A.R,
                           reinterpret_cast<const double2*>(W.scal + SC_RM_RE), W.red, 1, W.Om16, W.ORm, stream,
                           nullptr, nullptr, W.n_cu, 1, W.Om + A.N);
                if (e != hipSuccess) return e;
                hipLaunchKernelGGL(k_f_of, dim3(nblk(P)), dim3(256), 0, stream, P, A.mode, W.ORm, W.scal, W.F);
                hipLaunchKernelGGL(k_zdot, dim3(64), dim3(256), 0, stream, P, W.F, W.F, W.red, W.scal, 0);
                hipLaunchKernelGGL(k_sum_to, dim3(1), dim3(64), 0, stream, W.red, 64, W.scal, (int)SC_FF, 0);
            } else {
                e = run_ot(A.N, A.M, W.sig16, A.T, A.n, 0, 0, 1, nullptr, A.R, nullptr, W.red, 1, W.Om16, nullptr,
                           stream, nullptr, nullptr, W.n_cu, 0, W.Om + A.N);
                if (e != hipSuccess) return e;
            }
            const int nsplit = W.spart ? sbuild_splits(A.N, A.M, A.n, W.n_cu, W.nsplit_max) : 1;
            const int nsb = sbuild_border_splits(A.N, A.M, A.n, W.n_cu, W.nsb_max);
            e = launch_sbuild_mfma(A.N, A.M, P, A.samples, A.T, A.n, W.Om, W.Om16, W.S, A.prec, W.sb_kt, W.pack,
                                   W.pack_bytes, W.sb_order, W.sb_order_len,
                                   W.spart, nsplit, W.bx, W.bx_part, nsb, W.prof, stream);
        } else {
            // weighted (enumeration) sums: FP32 contraction on the vector units
            const int nt = (int)((P + SB_T - 1) / SB_T);
            const long ntri = (long)nt * (nt + 1) / 2;
            W.prof->begin(PROF_SBUILD, stream);
            hipLaunchKernelGGL(k_sbuild, dim3((unsigned)ntri), dim3(256), 0, stream, A.N, A.M, P, A.samples, A.T,
                               A.weights, A.n, W.Om, W.S, nt, W.scal,
                               A.solver == CRBM_SOLVER_CHOLESKY ? W.S64 : nullptr);
            W.prof->end(stream);
            e = hipGetLastError();
        }
        if (e != hipSuccess) return e;
    }

    if (A.solver == CRBM_SOLVER_CHOLESKY) {
        W.prof->begin(PROF_CHOLESKY, stream);
        e = launch_cholesky_solve(P, W.S, A.eps, W.F, W.S64, W.x, W.scal, A.weights != nullptr, stream);
        W.prof->end(stream);
        if (e != hipSuccess) return e;
        // residual of the double solve against the FP32-stored S
        hipLaunchKernelGGL(k_undone, dim3(1), dim3(64), 0, stream, W.scal);
    } else {
        hipLaunchKernelGGL(k_cg_init, dim3(nblk(P)), dim3(256), 0, stream, P, W.F, W.x, W.r, W.p);
        hipLaunchKernelGGL(k_cg_start, dim3(1), dim3(64), 0, stream, W.scal);
        W.prof->begin(PROF_CG, stream);
        // partials: W.red[0, 64) for p^H Ap, W.red[64, 64 + nblk(P)) for r^H r
        const int n_rr = (int)nblk(P);
        for (int it = 0; it < A.cg_maxit; ++it) {
            const int slot = (it & 1) ? (int)SC_RR1 : (int)SC_RR;
            e = apply_op(A, W, W.p, W.Ap, stream);
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL(k_zdot, dim3(64), dim3(256), 0, stream, P, W.p, W.Ap, W.red, W.scal, 1);
            hipLaunchKernelGGL(k_cg_xr, dim3(n_rr), dim3(256), 0, stream, P, W.x, W.r, W.p, W.Ap, W.red, W.red + 64,
                               W.scal, slot);
            hipLaunchKernelGGL(k_cg_check_p, dim3(n_rr), dim3(256), 0, stream, P, W.p, W.r, W.red + 64, n_rr, W.scal,
                               A.cg_tol, A.cg_maxit, it, slot);
        }
        W.prof->end(stream);
        hipLaunchKernelGGL(k_undone, dim3(1), dim3(64), 0, stream, W.scal);
    }
    // true residual |F - (S + eps) x|^2 in double
    e = apply_op(A, W, W.x, W.Ap, stream);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_resid, dim3(nblk(P)), dim3(256), 0, stream, P, W.F, W.Ap, W.r);
    hipLaunchKernelGGL(k_zdot, dim3(64), dim3(256), 0, stream, P, W.r, W.r, W.red, W.scal, 0);
    hipLaunchKernelGGL(k_sum_to, dim3(1), dim3(64), 0, stream, W.red, 64, W.scal, (int)SC_RESID, 0);
    hipLaunchKernelGGL(k_zdot, dim3(64), dim3(256), 0, stream, P, W.x, W.x, W.red, W.scal, 0);
    hipLaunchKernelGGL(k_sum_to, dim3(1), dim3(64), 0, stream, W.red, 64, W.scal, (int)SC_XX, 0);
    hipLaunchKernelGGL(k_update, dim3(nblk(P)), dim3(256), 0, stream, A.N, A.M, A.a, A.b, A.W, W.x, W.scal);
    if (A.stats) hipLaunchKernelGGL(k_stats, dim3(1), dim3(64), 0, stream, W.scal, A.stats);
    return hipGetLastError();
}

// ------------------------------------------------------------------ fidelity gradient
__global__ void k_loss(const float2* __restrict__ R, long n, double* __restrict__ loss) {
    __shared__ double sh[4];
    double acc = 0;
    for (long s = threadIdx.x; s < n; s += blockDim.x) {
        const double x = 1.0 - (double)R[s].x, y = -(double)R[s].y;
        acc += x * x + y * y;
    }
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) *loss = (sh[0] + sh[1] + sh[2] + sh[3]) / (double)n;
}

// the gradient from caller-chosen scratch: sig16 (n sig16_row(N) bytes) and the contraction's chunk planes
static hipError_t fidelity_grad_on(const GradArgs& A, int8_t* sig16, void* partial, int n_cu, Profiler* prof,
                                   hipStream_t stream) {
    if (A.grad) {
        pack_sig16(A.samples, A.n, A.N, sig16, stream);
        hipError_t e = run_ot(A.N, A.M, sig16, A.T, A.n, 3, 0, 1, nullptr, A.R, nullptr, partial, 0, A.grad, nullptr,
                              stream, nullptr, prof, n_cu);
        if (e != hipSuccess) return e;
    }
    if (A.loss) hipLaunchKernelGGL(k_loss, dim3(1), dim3(256), 0, stream, A.R, A.n, A.loss);
    return hipGetLastError();
}

hipError_t launch_fidelity_grad(const GradArgs& A, const SrWork& W, hipStream_t stream) {
    return fidelity_grad_on(A, W.sig16, W.red, W.n_cu, W.prof, stream);
}

// Scratch of the gradient for n samples, laid out as [sigma~ rows | 256-byte alignment | chunk planes of one
// coefficient, 2 (N + 1)(M + 1) floats per sample chunk]; the chunk count depends on n only.
size_t fidelity_grad_scratch_bytes(int N, int M, long n) {
    long chunk;
    int n_chunks;
    ot_chunking(n, chunk, n_chunks);
    const size_t rows = ((size_t)n * (size_t)sig16_row(N) + 255) / 256 * 256;
    return rows + (size_t)n_chunks * 2 * (size_t)(N + 1) * (size_t)(M + 1) * sizeof(float);
}

hipError_t launch_fidelity_grad_scratch(const GradArgs& A, void* scratch, int n_cu, hipStream_t stream) {
    int8_t* sig16 = static_cast<int8_t*>(scratch);
    const size_t rows = ((size_t)A.n * (size_t)sig16_row(A.N) + 255) / 256 * 256;
    return fidelity_grad_on(A, sig16, static_cast<unsigned char*>(scratch) + rows, n_cu, nullptr, stream);
}

}  // namespace crbm
