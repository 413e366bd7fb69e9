// Moment correction, Krylov continued fraction and spectral reconstruction.
//
// Basis.  t_0 = S^z_q psi_gs and t_n = beta_n t~_n (n = 1..K-1), sampled over
// s ~ |psi_gs|^2 through the ratios B_n(s) = t_n(s)/psi_gs(s) and
// HB_n(s) = (H t_n)(s)/psi_gs(s) (App. A).  The per-order columns B_n, HB_n
// are produced by the existing theta / local-energy / ratio kernels and packed
// here; the overlap and Hamiltonian matrices (Sec. IV)
//   G_nm = <conj(B_n) B_m>,   H_nm = <conj(B_n) HB_m>
// are one tall-skinny product [K x n] x [n x K] each, accumulated in double
// (products of binary32 values are exact in binary64).
//
// Small dense work (K <= 256) runs in single-workgroup kernels in double:
// Cholesky of G, the Chebyshev recursion inside the span (Sec. IV), and a
// Lanczos tridiagonalisation of the projected Hamiltonian for the continued
// fraction (Sec. V).  The spectra on a frequency grid are one thread per
// frequency: Eq. (Aw) with the Jackson factors of Sec. VI, and the continued
// fraction evaluated from its last level upwards.
#include <hip/hip_runtime.h>

#include "../../include/chebrbm.h"
#include "device.hpp"
#include "internal.hpp"

namespace crbm {

// ------------------------------------------------------------------ basis columns
// Bcol[s] = B(s);  HBcol[s] = B(s) * loc(s) (mul = 1: loc = E_loc of t~_n) or loc(s) (mul = 0: order 0)
__global__ __launch_bounds__(256) void k_basis_pack(long n, const double2* __restrict__ B, const float2* __restrict__ loc,
                                                    int mul, float2* __restrict__ Bcol, float2* __restrict__ HBcol) {
    const long s = (long)blockIdx.x * 256 + threadIdx.x;
    if (s >= n) return;
    const double2 b = B[s];
    const float2 bf = make_float2((float)b.x, (float)b.y);
    Bcol[s] = bf;
    HBcol[s] = mul ? cmul(bf, loc[s]) : loc[s];
}

hipError_t launch_basis_pack(long n, const double2* B, const float2* loc, int mul, float2* Bcol, float2* HBcol,
                             hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_basis_pack, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, n, B, loc, mul, Bcol,
                       HBcol);
    return hipGetLastError();
}

// ------------------------------------------------------------------ Gram products
// Block (x, y): sample chunk x, output tile y = (tk, tl) of 32 x 32 entries of both G and H.
// Thread t owns row k0 + (t >> 3) and columns l0 + 4 (t & 7) + [0, 4).
constexpr int GR_T = 32, GR_S = 32;

__global__ __launch_bounds__(256) void k_gram2(int K, long n, long chunk, const float2* __restrict__ Bm,
                                               const float2* __restrict__ HBm, const double* __restrict__ w,
                                               double wdef, double2* __restrict__ partial) {
    __shared__ float2 sk[GR_S][GR_T + 1];
    __shared__ float2 sl[GR_S][GR_T + 1];
    __shared__ float2 sh[GR_S][GR_T + 1];
    __shared__ double sw[GR_S];
    const int nt = (K + GR_T - 1) / GR_T;
    const int tk = blockIdx.y / nt, tl = blockIdx.y % nt;
    const int k0 = tk * GR_T, l0 = tl * GR_T;
    const int tid = threadIdx.x;
    const int kr = tid >> 3, lc = (tid & 7) * 4;
    const long s_begin = (long)blockIdx.x * chunk;
    const long s_end = min(n, s_begin + chunk);
    double2 g[4], h[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) { g[j] = make_double2(0.0, 0.0); h[j] = make_double2(0.0, 0.0); }
    for (long sb = s_begin; sb < s_end; sb += GR_S) {
        for (int e = tid; e < GR_S * GR_T; e += 256) {
            const int row = e / GR_S, ss = e % GR_S;
            const long s = sb + ss;
            const bool vs = s < s_end;
            const int k = k0 + row, l = l0 + row;
            sk[ss][row] = (vs && k < K) ? Bm[(long)k * n + s] : make_float2(0.f, 0.f);
            sl[ss][row] = (vs && l < K) ? Bm[(long)l * n + s] : make_float2(0.f, 0.f);
            sh[ss][row] = (vs && l < K) ? HBm[(long)l * n + s] : make_float2(0.f, 0.f);
        }
        if (tid < GR_S) {
            const long s = sb + tid;
            sw[tid] = s < s_end ? (w ? w[s] : wdef) : 0.0;
        }
        __syncthreads();
#pragma unroll 4
        for (int ss = 0; ss < GR_S; ++ss) {
            const float2 bk = sk[ss][kr];
            const double ws = sw[ss];
            const double ax = ws * (double)bk.x, ay = -ws * (double)bk.y;     // w conj(B_k)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float2 bl = sl[ss][lc + j], hl = sh[ss][lc + j];
                g[j].x = fma(ax, (double)bl.x, fma(-ay, (double)bl.y, g[j].x));
                g[j].y = fma(ax, (double)bl.y, fma(ay, (double)bl.x, g[j].y));
                h[j].x = fma(ax, (double)hl.x, fma(-ay, (double)hl.y, h[j].x));
                h[j].y = fma(ax, (double)hl.y, fma(ay, (double)hl.x, h[j].y));
            }
        }
        __syncthreads();
    }
    double2* out = partial + ((long)blockIdx.x * gridDim.y + blockIdx.y) * (2 * GR_T * GR_T);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        out[kr * GR_T + lc + j] = g[j];
        out[GR_T * GR_T + kr * GR_T + lc + j] = h[j];
    }
}

// G[k][l], H[k][l] = sum over chunks (in chunk order) of the tile partials (added to G, H if accumulate)
__global__ __launch_bounds__(256) void k_gram_final(int K, int n_chunks, int tiles, const double2* __restrict__ partial,
                                                    int accumulate, double2* __restrict__ G,
                                                    double2* __restrict__ H) {
    const long idx = (long)blockIdx.x * 256 + threadIdx.x;
    const long per = 2L * GR_T * GR_T;
    if (idx >= (long)tiles * per) return;
    const int tile = (int)(idx / per);
    const int r = (int)(idx % per);
    const int which = r / (GR_T * GR_T);
    const int kr = (r % (GR_T * GR_T)) / GR_T, lc = r % GR_T;
    const int nt = (K + GR_T - 1) / GR_T;
    const int k = (tile / nt) * GR_T + kr, l = (tile % nt) * GR_T + lc;
    if (k >= K || l >= K) return;
    double2 acc = make_double2(0.0, 0.0);
    for (int c = 0; c < n_chunks; ++c) acc = zadd(acc, partial[((long)c * tiles + tile) * per + r]);
    double2* dst = (which ? H : G) + (long)k * K + l;
    *dst = accumulate ? zadd(*dst, acc) : acc;
}

long gram_partial_len(int K) {
    const int nt = (K + GR_T - 1) / GR_T;
    const int tiles = nt * nt;
    const int nbx = tiles >= 1024 ? 1 : 1024 / tiles;
    return (long)nbx * tiles * 2 * GR_T * GR_T;
}

// columns Bm[k][n], HBm[k][n]; sample weights w[s] or wdef; G, H = (accumulate ? G, H + : ) the products
hipError_t launch_gram2(int K, long n, const float2* Bm, const float2* HBm, const double* w, double wdef,
                        double2* partial, double2* G, double2* H, int accumulate, hipStream_t stream) {
    const int nt = (K + GR_T - 1) / GR_T;
    const int tiles = nt * nt;
    int nbx = tiles >= 1024 ? 1 : 1024 / tiles;
    long chunk = (n + nbx - 1) / nbx;
    chunk = ((chunk + GR_S - 1) / GR_S) * GR_S;
    nbx = (int)((n + chunk - 1) / chunk);
    hipLaunchKernelGGL(k_gram2, dim3(nbx, tiles), dim3(256), 0, stream, K, n, chunk, Bm, HBm, w, wdef, partial);
    const long total = (long)tiles * 2 * GR_T * GR_T;
    hipLaunchKernelGGL(k_gram_final, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, stream, K, nbx, tiles,
                       partial, accumulate, G, H);
    return hipGetLastError();
}

// ------------------------------------------------------------------ symmetry projection (App. A)
// Group elements g = T_m R^rot, index gi = (m1 + Lx m2) nrot + rot, with R(x, y) = (L-1-y, x) on the
// L x L lattice (nrot = 4) or translations only (nrot = 1).  An element acts on configurations as
// (s o g)_r = s_{g(r)}, so that <s|g|t> = t(s o g).
__device__ __forceinline__ int sym_map(int kind, int Lx, int Ly, int m1, int m2, int rot, int r) {
    int x = kind == 0 ? r : r % Lx, y = kind == 0 ? 0 : r / Lx;
    for (int q = 0; q < rot; ++q) {
        const int nx = Lx - 1 - y;
        y = x;
        x = nx;
    }
    x += m1;
    if (x >= Lx) x -= Lx;
    if (kind == 0) return x;
    y += m2;
    if (y >= Ly) y -= Ly;
    return x + Lx * y;
}

// img[(s ng + gi) N + r] = sig[s N + g(r)] for the c samples of a chunk
__global__ __launch_bounds__(256) void k_sym_images(const int8_t* __restrict__ sig, long c, int N, int kind, int Lx,
                                                    int Ly, int nrot, int8_t* __restrict__ img) {
    const long ng = (long)N * nrot;
    const long idx = (long)blockIdx.x * 256 + threadIdx.x;
    if (idx >= c * ng * N) return;
    const int r = (int)(idx % N);
    const long row = idx / N;
    const int gi = (int)(row % ng);
    const long s = row / ng;
    const int rot = gi % nrot, m = gi / nrot;
    const int m1 = m % Lx, m2 = m / Lx;
    img[idx] = sig[s * N + sym_map(kind, Lx, Ly, m1, m2, rot, r)];
}

// Per image row (s, g):  order 0: B = (s o g)_0 / 2 psi_gs(s o g)/psi_gs(s), HB = ((H t_000)(s o g)/psi_gs(s o g))
// psi_gs(s o g)/psi_gs(s);  order n: B = beta_n t_n(s o g)/psi_gs(s), HB = B E_loc[t_n](s o g).
// lt: log amplitude of the order's RBM on the images; el: its local quantity there; lg: log psi_gs(s).
__global__ __launch_bounds__(256) void k_sym_combine(long rows, int ng, int N, const int8_t* __restrict__ img,
                                                     int order0, const float2* __restrict__ lt,
                                                     const float2* __restrict__ el, const float2* __restrict__ lg,
                                                     const double2* __restrict__ beta, float2* __restrict__ B,
                                                     float2* __restrict__ HB) {
    const long row = (long)blockIdx.x * 256 + threadIdx.x;
    if (row >= rows) return;
    const long s = row / ng;
    const float2 r = cexpf(csub(lt[row], lg[s]));
    if (order0) {
        B[row] = cscale(r, 0.5f * (float)img[row * N]);
        HB[row] = cmul(r, el[row]);
    } else {
        const float2 b = cmul(make_float2((float)beta->x, (float)beta->y), r);
        B[row] = b;
        HB[row] = cmul(b, el[row]);
    }
}

// Bt[(k K + n) c + s] = N^{-1/2} (1/nrot) sum_m e^{-i k.m} sum_rot B[n][(s ng + g(m + d_rot, rot))],
// d = (0,0), (1,0), (1,1), (0,1); likewise HBt.  One workgroup per (s, n); k = k1 + Lx k2 for all N momenta.
__global__ __launch_bounds__(256) void k_sym_dft(long c, int K, int N, int kind, int Lx, int Ly, int nrot,
                                                 const float2* __restrict__ B, const float2* __restrict__ HB,
                                                 float2* __restrict__ Bt, float2* __restrict__ HBt) {
    __shared__ float2 sb[1024], sh[1024];
    __shared__ float2 twx[256], twy[256];
    const long s = blockIdx.x;
    const int n = blockIdx.y;
    const int ng = N * nrot;
    const int L2 = kind == 0 ? 1 : Ly;
    const long base = (long)n * c * ng + s * ng;
    for (int e = threadIdx.x; e < ng; e += 256) { sb[e] = B[base + e]; sh[e] = HB[base + e]; }
    for (int e = threadIdx.x; e < Lx; e += 256) {
        float sn, cs;
        sincospif(-2.0f * (float)e / (float)Lx, &sn, &cs);
        twx[e] = make_float2(cs, sn);
    }
    for (int e = threadIdx.x; e < L2; e += 256) {
        float sn, cs;
        sincospif(-2.0f * (float)e / (float)L2, &sn, &cs);
        twy[e] = make_float2(cs, sn);
    }
    __syncthreads();
    const int off1[4] = {0, 1, 1, 0}, off2[4] = {0, 0, 1, 1};
    const float norm = rsqrtf((float)N) / (float)nrot;
    for (int kk = threadIdx.x; kk < N; kk += 256) {
        const int k1 = kk % Lx, k2 = kk / Lx;
        float2 ab = make_float2(0.f, 0.f), ah = make_float2(0.f, 0.f);
        for (int m2 = 0; m2 < L2; ++m2)
            for (int m1 = 0; m1 < Lx; ++m1) {
                const float2 tw = cmul(twx[(k1 * m1) % Lx], twy[(k2 * m2) % L2]);
                float2 vb = make_float2(0.f, 0.f), vh = make_float2(0.f, 0.f);
                for (int rot = 0; rot < nrot; ++rot) {
                    int a1 = m1 + off1[rot], a2 = m2 + off2[rot];
                    if (a1 >= Lx) a1 -= Lx;
                    if (a2 >= L2) a2 -= L2;
                    const int gi = (a1 + Lx * a2) * nrot + rot;
                    vb = cadd(vb, sb[gi]);
                    vh = cadd(vh, sh[gi]);
                }
                ab = cadd(ab, cmul(tw, vb));
                ah = cadd(ah, cmul(tw, vh));
            }
        Bt[((long)kk * K + n) * c + s] = cscale(ab, norm);
        HBt[((long)kk * K + n) * c + s] = cscale(ah, norm);
    }
}

hipError_t launch_sym_images(const int8_t* sig, long c, int N, int kind, int Lx, int Ly, int nrot, int8_t* img,
                             hipStream_t stream) {
    const long total = c * (long)N * nrot * N;
    hipLaunchKernelGGL(k_sym_images, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, stream, sig, c, N, kind, Lx,
                       Ly, nrot, img);
    return hipGetLastError();
}

hipError_t launch_sym_combine(long rows, int ng, int N, const int8_t* img, int order0, const float2* lt,
                              const float2* el, const float2* lg, const double2* beta, float2* B, float2* HB,
                              hipStream_t stream) {
    hipLaunchKernelGGL(k_sym_combine, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, stream, rows, ng, N, img,
                       order0, lt, el, lg, beta, B, HB);
    return hipGetLastError();
}

hipError_t launch_sym_dft(long c, int K, int N, int kind, int Lx, int Ly, int nrot, const float2* B, const float2* HB,
                          float2* Bt, float2* HBt, hipStream_t stream) {
    hipLaunchKernelGGL(k_sym_dft, dim3((unsigned)c, (unsigned)K), dim3(256), 0, stream, c, K, N, kind, Lx, Ly, nrot,
                       B, HB, Bt, HBt);
    return hipGetLastError();
}

// ------------------------------------------------------------------ single-workgroup dense work
constexpr int SM_THREADS = 256;

__device__ __forceinline__ double2 zconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 zscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }

// sum over the workgroup (256 threads); every thread gets the result
__device__ double block_sum(double v, double* red) {
    v = wave_sum(v);
    const int wv = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[wv] = v;
    __syncthreads();
    return red[0] + red[1] + red[2] + red[3];
}
__device__ double2 block_zsum(double2 v, double* red) {
    const double x = block_sum(v.x, red);
    const double y = block_sum(v.y, red + 4);
    return make_double2(x, y);
}

// L (row-major, lower triangle) <- Cholesky factor of the Hermitian part of G.
// Returns false (same value in every thread) if a pivot is not positive and finite.
__device__ bool block_cholesky(int K, const double2* __restrict__ G, double2* __restrict__ L, double* piv_min,
                               double* piv_max, int* s_fail) {
    for (long e = threadIdx.x; e < (long)K * K; e += SM_THREADS) {
        const int i = (int)(e / K), j = (int)(e % K);
        L[e] = (j <= i) ? zscale(zadd(G[(long)i * K + j], zconj(G[(long)j * K + i])), 0.5) : make_double2(0.0, 0.0);
    }
    if (threadIdx.x == 0) { *s_fail = 0; *piv_min = 1e300; *piv_max = 0.0; }
    __syncthreads();
    for (int j = 0; j < K; ++j) {
        if (threadIdx.x == 0) {
            const double d = L[(long)j * K + j].x;
            if (!(d > 0.0) || !isfinite(d)) *s_fail = 1;
            else {
                L[(long)j * K + j] = make_double2(sqrt(d), 0.0);
                *piv_min = fmin(*piv_min, d);
                *piv_max = fmax(*piv_max, d);
            }
        }
        __syncthreads();
        if (*s_fail) return false;
        const double inv = 1.0 / L[(long)j * K + j].x;
        for (int i = j + 1 + threadIdx.x; i < K; i += SM_THREADS) L[(long)i * K + j] = zscale(L[(long)i * K + j], inv);
        __syncthreads();
        // trailing update of the lower triangle: L[i][k] -= L[i][j] conj(L[k][j]), j < k <= i
        const int m = K - j - 1;
        for (long e = threadIdx.x; e < (long)m * m; e += SM_THREADS) {
            const int i = j + 1 + (int)(e / m), k = j + 1 + (int)(e % m);
            if (k <= i) L[(long)i * K + k] = zsub(L[(long)i * K + k], zmul(L[(long)i * K + j], zconj(L[(long)k * K + j])));
        }
        __syncthreads();
    }
    return true;
}

// In-place solve L y = x (forward) for a vector held by one thread (strided by `st` in memory).
__device__ void fwd_solve(int K, const double2* __restrict__ L, double2* x, long st) {
    for (int i = 0; i < K; ++i) {
        double2 acc = x[i * st];
        for (int j = 0; j < i; ++j) acc = zsub(acc, zmul(L[(long)i * K + j], x[j * st]));
        x[i * st] = zscale(acc, 1.0 / L[(long)i * K + i].x);
    }
}
// In-place solve L^H y = x (backward).
__device__ void bwd_solve(int K, const double2* __restrict__ L, double2* x, long st) {
    for (int i = K - 1; i >= 0; --i) {
        double2 acc = x[i * st];
        for (int j = i + 1; j < K; ++j) acc = zsub(acc, zmul(zconj(L[(long)j * K + i]), x[j * st]));
        x[i * st] = zscale(acc, 1.0 / L[(long)i * K + i].x);
    }
}

// Corrected moments (Sec. IV).  Work: L [K*K], Xc [K*K] (column-major G^{-1} H'), v [3K].
// info: [0] flags, [1] max_n |mu_n| / mu_0, [2] min pivot / max pivot of the Cholesky factorisation.
__global__ __launch_bounds__(SM_THREADS) void k_correct(int K, const double2* __restrict__ G,
                                                        const double2* __restrict__ H, double E_c, double W_scale,
                                                        int n_out, double2* __restrict__ L, double2* __restrict__ Xc,
                                                        double2* __restrict__ v, double* __restrict__ mu,
                                                        double* __restrict__ info) {
    __shared__ double red[8];
    __shared__ double pmin, pmax;
    __shared__ int fail;
    if (!block_cholesky(K, G, L, &pmin, &pmax, &fail)) {
        if (threadIdx.x == 0) { info[0] = CRBM_FLAG_CHOLESKY_FAIL; info[1] = 0.0; info[2] = 0.0; }
        for (int n = threadIdx.x; n < n_out; n += SM_THREADS) mu[n] = 0.0;
        return;
    }
    // Xc[:, c] = G^{-1} H'[:, c], H' = (herm(H) - E_c herm(G)) / W_scale; column c is thread c's
    const double invW = 1.0 / W_scale;
    for (int c = threadIdx.x; c < K; c += SM_THREADS) {
        double2* x = Xc + (long)c * K;
        for (int i = 0; i < K; ++i) {
            const double2 hh = zscale(zadd(H[(long)i * K + c], zconj(H[(long)c * K + i])), 0.5);
            const double2 gh = zscale(zadd(G[(long)i * K + c], zconj(G[(long)c * K + i])), 0.5);
            x[i] = zscale(zsub(hh, zscale(gh, E_c)), invW);
        }
        fwd_solve(K, L, x, 1);
        bwd_solve(K, L, x, 1);
    }
    __syncthreads();
    // recursion c_0 = e_0, c_1 = X e_0, c_{n+1} = 2 X c_n - c_{n-1};  mu_n = Re sum_l herm(G)_{0l} c_{ln}
    double2* cp = v;
    double2* cc = v + K;
    double2* cn = v + 2 * K;
    const double mu0 = G[0].x;
    double growth = 1.0;
    for (int i = threadIdx.x; i < K; i += SM_THREADS) {
        cp[i] = make_double2(i == 0 ? 1.0 : 0.0, 0.0);
        cc[i] = Xc[i];
    }
    if (threadIdx.x == 0) mu[0] = mu0;
    __syncthreads();
    for (int n = 1; n < n_out; ++n) {
        double part = 0.0;
        for (int l = threadIdx.x; l < K; l += SM_THREADS) {
            const double2 g0l = zscale(zadd(G[l], zconj(G[(long)l * K])), 0.5);
            part += g0l.x * cc[l].x - g0l.y * cc[l].y;
        }
        const double m = block_sum(part, red);
        if (threadIdx.x == 0) mu[n] = m;
        growth = fmax(growth, fabs(m) / fabs(mu0));
        if (n + 1 < n_out) {
            for (int i = threadIdx.x; i < K; i += SM_THREADS) {
                double2 acc = make_double2(0.0, 0.0);
                for (int l = 0; l < K; ++l) acc = zadd(acc, zmul(Xc[(long)l * K + i], cc[l]));
                cn[i] = zsub(zscale(acc, 2.0), cp[i]);
            }
            __syncthreads();
            double2* t = cp; cp = cc; cc = cn; cn = t;
        }
    }
    if (threadIdx.x == 0) {
        info[0] = 0.0;
        info[1] = growth;
        info[2] = pmin / pmax;
    }
}

// Lanczos tridiagonalisation of the projected Hamiltonian (Sec. V).  With G = L L^H the basis
// L^{-H}-orthonormalised has Hamiltonian Hhat = L^{-1} herm(H) L^{-H}, and t_0 becomes
// sqrt(G_00) e_0.  Plain Lanczos from e_0 with full re-orthogonalisation (two passes).
// Work: L [K*K], Y [K*K], Q [K*K] (column j = Lanczos vector j), w [K].
// a_out[j] = <q_j|Hhat|q_j>, b2_out[0] = G_00, b2_out[j] = b_j^2 (j >= 1); info: [0] flags, [1] steps done.
__global__ __launch_bounds__(SM_THREADS) void k_lanczos(int K, const double2* __restrict__ G,
                                                        const double2* __restrict__ H, int n_steps,
                                                        double2* __restrict__ L, double2* __restrict__ Y,
                                                        double2* __restrict__ Q, double2* __restrict__ wv,
                                                        double* __restrict__ a_out, double* __restrict__ b2_out,
                                                        double* __restrict__ info) {
    __shared__ double red[8];
    __shared__ double pmin, pmax;
    __shared__ int fail;
    if (!block_cholesky(K, G, L, &pmin, &pmax, &fail)) {
        if (threadIdx.x == 0) { info[0] = CRBM_FLAG_CHOLESKY_FAIL; info[1] = 0.0; }
        return;
    }
    // Y (column-major): column c = L^{-1} herm(H)[:, c]
    for (int c = threadIdx.x; c < K; c += SM_THREADS) {
        double2* y = Y + (long)c * K;
        for (int i = 0; i < K; ++i)
            y[i] = zscale(zadd(H[(long)i * K + c], zconj(H[(long)c * K + i])), 0.5);
        fwd_solve(K, L, y, 1);
    }
    __syncthreads();
    // Hhat = L^{-1} Y^H: column c from the conjugated row c of Y, i.e. conj(Y[c][i]) = conj(Ycol_i[c]);
    // stored column-major in Q temporarily, then copied into Y (Hhat, column-major).
    for (int c = threadIdx.x; c < K; c += SM_THREADS) {
        double2* z = Q + (long)c * K;
        for (int i = 0; i < K; ++i) z[i] = zconj(Y[(long)i * K + c]);
        fwd_solve(K, L, z, 1);
    }
    __syncthreads();
    for (long e = threadIdx.x; e < (long)K * K; e += SM_THREADS) Y[e] = Q[e];
    __syncthreads();
    // Hermitian part: Hhat <- (Hhat + Hhat^H)/2, in place over the pairs (i, c), i <= c
    for (long e = threadIdx.x; e < (long)K * K; e += SM_THREADS) {
        const int c = (int)(e / K), i = (int)(e % K);
        if (i <= c) {
            const double2 x = Y[(long)c * K + i], y = Y[(long)i * K + c];
            const double2 m = zscale(zadd(x, zconj(y)), 0.5);
            Y[(long)c * K + i] = m;
            Y[(long)i * K + c] = zconj(m);
        }
    }
    __syncthreads();
    for (long e = threadIdx.x; e < (long)K * K; e += SM_THREADS) Q[e] = make_double2(0.0, 0.0);
    __syncthreads();
    if (threadIdx.x == 0) { Q[0] = make_double2(1.0, 0.0); b2_out[0] = G[0].x; }
    // scale of Hhat for the breakdown test
    double fro = 0.0;
    for (long e = threadIdx.x; e < (long)K * K; e += SM_THREADS) fro += Y[e].x * Y[e].x + Y[e].y * Y[e].y;
    const double hnorm = sqrt(block_sum(fro, red));
    int done = 0;
    double b_prev = 0.0;
    for (int j = 0; j < n_steps; ++j) {
        const double2* q = Q + (long)j * K;
        // w = Hhat q_j  (thread i: row i = sum_c Hhat[i][c] q[c], Hhat column-major)
        for (int i = threadIdx.x; i < K; i += SM_THREADS) {
            double2 acc = make_double2(0.0, 0.0);
            for (int c = 0; c < K; ++c) acc = zadd(acc, zmul(Y[(long)c * K + i], q[c]));
            wv[i] = acc;
        }
        __syncthreads();
        double part = 0.0;
        for (int i = threadIdx.x; i < K; i += SM_THREADS) part += q[i].x * wv[i].x + q[i].y * wv[i].y;
        const double a = block_sum(part, red);
        if (threadIdx.x == 0) a_out[j] = a;
        for (int i = threadIdx.x; i < K; i += SM_THREADS) {
            double2 x = zsub(wv[i], zscale(q[i], a));
            if (j > 0) x = zsub(x, zscale(Q[(long)(j - 1) * K + i], b_prev));
            wv[i] = x;
        }
        __syncthreads();
        done = j + 1;
        if (j + 1 >= n_steps || j + 1 >= K) break;
        for (int pass = 0; pass < 2; ++pass) {
            for (int r = 0; r <= j; ++r) {
                const double2* qr = Q + (long)r * K;
                double2 p = make_double2(0.0, 0.0);
                for (int i = threadIdx.x; i < K; i += SM_THREADS) p = zadd(p, zmul(zconj(qr[i]), wv[i]));
                const double2 d = block_zsum(p, red);
                for (int i = threadIdx.x; i < K; i += SM_THREADS) wv[i] = zsub(wv[i], zmul(d, qr[i]));
                __syncthreads();
            }
        }
        double nn = 0.0;
        for (int i = threadIdx.x; i < K; i += SM_THREADS) nn += wv[i].x * wv[i].x + wv[i].y * wv[i].y;
        const double b2 = block_sum(nn, red);
        const double b = sqrt(b2);
        if (!(b > 1e-13 * hnorm)) break;          // invariant subspace reached: the fraction terminates
        if (threadIdx.x == 0) b2_out[j + 1] = b2;
        double2* qn = Q + (long)(j + 1) * K;
        for (int i = threadIdx.x; i < K; i += SM_THREADS) qn[i] = zscale(wv[i], 1.0 / b);
        b_prev = b;
        __syncthreads();
    }
    if (threadIdx.x == 0) { info[0] = 0.0; info[1] = (double)done; }
}

hipError_t launch_correct(int K, const double2* G, const double2* H, double E_c, double W_scale, int n_out,
                          double2* work, double* mu, double* info, hipStream_t stream) {
    double2* L = work;
    double2* X = work + (long)K * K;
    double2* v = work + 2L * K * K;
    hipLaunchKernelGGL(k_correct, dim3(1), dim3(SM_THREADS), 0, stream, K, G, H, E_c, W_scale, n_out, L, X, v, mu, info);
    return hipGetLastError();
}

hipError_t launch_lanczos(int K, const double2* G, const double2* H, int n_steps, double2* work, double* a, double* b2,
                          double* info, hipStream_t stream) {
    double2* L = work;
    double2* Y = work + (long)K * K;
    double2* Q = work + 2L * K * K;
    double2* w = work + 3L * K * K;
    hipLaunchKernelGGL(k_lanczos, dim3(1), dim3(SM_THREADS), 0, stream, K, G, H, n_steps, L, Y, Q, w, a, b2, info);
    return hipGetLastError();
}

// ------------------------------------------------------------------ spectra on a grid
// Eq. (Aw): A = [g_0 mu_0 + 2 sum g_n mu_n T_n(x)] / (pi W_scale sqrt(1 - x^2)), x = (E0 + omega - E_c)/W_scale,
// T_n by the three-term recursion; g_n the Jackson factors (or 1).  Zero for |x| >= 1.
__global__ __launch_bounds__(256) void k_spec_kpm(const double* __restrict__ mu, int n_mom, int jackson, double E0,
                                                  double E_c, double W_scale, const double* __restrict__ omega,
                                                  int n_w, double* __restrict__ A) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n_w) return;
    const double x = (E0 + omega[i] - E_c) / W_scale;
    if (!(fabs(x) < 1.0)) { A[i] = 0.0; return; }
    const double N1 = (double)(n_mom + 1);
    const double ang = M_PI / N1;
    const double cot = cos(ang) / sin(ang);
    double tm = 1.0, tc = x;
    double acc = mu[0];
    for (int n = 1; n < n_mom; ++n) {
        const double g = jackson ? ((N1 - n) * cos(ang * n) + sin(ang * n) * cot) / N1 : 1.0;
        acc += 2.0 * g * mu[n] * tc;
        const double tn = 2.0 * x * tc - tm;
        tm = tc;
        tc = tn;
    }
    A[i] = acc / (M_PI * W_scale * sqrt(1.0 - x * x));
}

// A = -(1/pi) Im [ b2_0 / (z - a_0 - b2_1 / (z - a_1 - ... - b2_{m-1} / (z - a_{m-1}))) ], z = omega + E0 + i eta
__global__ __launch_bounds__(256) void k_spec_cf(const double* __restrict__ a, const double* __restrict__ b2, int m,
                                                 double E0, double eta, const double* __restrict__ omega, int n_w,
                                                 double* __restrict__ A) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n_w) return;
    const double2 z = make_double2(omega[i] + E0, eta);
    double2 d = make_double2(z.x - a[m - 1], z.y);
    for (int j = m - 2; j >= 0; --j) {
        const double2 q = zdiv(make_double2(b2[j + 1], 0.0), d);
        d = make_double2(z.x - a[j] - q.x, z.y - q.y);
    }
    const double2 g = zdiv(make_double2(b2[0], 0.0), d);
    A[i] = -g.y / M_PI;
}

hipError_t launch_spec_kpm(const double* mu, int n_mom, int jackson, double E0, double E_c, double W_scale,
                           const double* omega, int n_w, double* A, hipStream_t stream) {
    hipLaunchKernelGGL(k_spec_kpm, dim3((n_w + 255) / 256), dim3(256), 0, stream, mu, n_mom, jackson, E0, E_c, W_scale,
                       omega, n_w, A);
    return hipGetLastError();
}

hipError_t launch_spec_cf(const double* a, const double* b2, int m, double E0, double eta, const double* omega,
                          int n_w, double* A, hipStream_t stream) {
    hipLaunchKernelGGL(k_spec_cf, dim3((n_w + 255) / 256), dim3(256), 0, stream, a, b2, m, E0, eta, omega, n_w, A);
    return hipGetLastError();
}

}  // namespace crbm
