// Dense Hermitian positive-definite solve (S + eps I) x = F in double precision
// by a Cholesky factorisation L L^H followed by two triangular solves.  Used for
// the natural-gradient system of Sec. III when P is a few thousand (the
// factorisation costs P^3/3 complex multiply-adds).
//
// Right-looking and blocked in panels of CH_NB = 64 columns, per panel k:
//   1. the diagonal block A_kk is factored in LDS by one workgroup;
//   2. the rows below solve L_ik L_kk^H = A_ik, one wave per row (the lanes hold
//      the 64 unknowns of the row, the substitution runs along the columns);
//   3. the trailing lower triangle is updated, A_ij -= L_ik L_jk^H (i >= j), in
//      32 x 32 output tiles with both 32 x 64 panels staged in LDS.
// The triangular solves run by blocks of 64 rows: one wave substitutes in the
// diagonal block, a wide kernel applies the block to the rest of the vector.
// Everything is in double, in a fixed order.
#include "../../include/chebrbm.h"
#include "device.hpp"
#include "internal.hpp"

namespace crbm {

enum { SC_FLAGS_SLOT = 15 };   // must match the scalar layout of the step driver
constexpr int CH_NB = 64;      // panel width
constexpr int CH_T = 32;       // trailing-update tile

// the value of v in lane m (m wave-uniform), through scalar registers
__device__ __forceinline__ double lane_value(double v, int m) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, m), hi = __builtin_amdgcn_readlane((int)(b >> 32), m);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

__device__ __forceinline__ bool chol_failed(const double* sc) {
    return ((int)sc[SC_FLAGS_SLOT] & CRBM_FLAG_CHOLESKY_FAIL) != 0;
}

// A64 = S + eps I (lower triangle used); S == null: A64 already holds S in double, only the shift is added
__global__ __launch_bounds__(256) void k_chol_load(long P, const float2* __restrict__ S, double eps,
                                                   double2* __restrict__ A) {
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= P * P) return;
    const long i = idx / P, j = idx % P;
    if (!S) {
        if (i == j) A[idx].x += eps;
        return;
    }
    const float2 v = S[idx];
    A[idx] = make_double2((double)v.x + (i == j ? eps : 0.0), (double)v.y);
}

// 1. L_kk of the diagonal block [k0, k0 + nb)^2 in LDS (one workgroup of 1024 threads, a 32 x 32 grid over
//    rows and columns, four waves per SIMD to overlap their LDS latencies).  Column j: every thread reads the
//    pivot d = L_jj (final since the last barrier, so all take the same decision) and updates its share of
//    the trailing lower triangle with the column scaled by 1 / sqrt(d) on the fly; after one barrier the
//    column itself is scaled.  The next column reads column j + 1 and its own trailing block only, so one
//    barrier per column suffices.
__global__ __launch_bounds__(1024) void k_chol_diagblock(long P, long k0, int nb, double2* __restrict__ A,
                                                         double* __restrict__ sc) {
    __shared__ double2 L[CH_NB][CH_NB + 1];
    if (chol_failed(sc)) return;
    const int tid = threadIdx.x, tx = tid & 31, ty = tid >> 5;
    for (int i = ty; i < nb; i += 32)
        for (int j = tx; j < nb; j += 32) L[i][j] = (j <= i) ? A[(k0 + i) * P + k0 + j] : make_double2(0.0, 0.0);
    __syncthreads();
    bool fail = false;
    for (int j = 0; j < nb; ++j) {
        const double d = L[j][j].x;
        if (!(d > 0.0) || !isfinite(d)) {
            fail = true;
            break;
        }
        const double s = sqrt(d), inv = 1.0 / s;
        double2 b[2];                                  // L_lj / s for this thread's columns l
#pragma unroll
        for (int m = 0; m < 2; ++m) {
            const int l = j + 1 + tx + 32 * m;
            b[m] = l < nb ? make_double2(L[l][j].x * inv, L[l][j].y * inv) : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            const int i = j + 1 + ty + 32 * p;
            if (i >= nb) break;
            const double2 a = make_double2(L[i][j].x * inv, L[i][j].y * inv);
#pragma unroll
            for (int m = 0; m < 2; ++m) {
                const int l = j + 1 + tx + 32 * m;
                if (l <= i) {                          // L_il -= L_ij conj(L_lj)
                    L[i][l].x -= a.x * b[m].x + a.y * b[m].y;
                    L[i][l].y -= a.y * b[m].x - a.x * b[m].y;
                }
            }
        }
        __syncthreads();
        if (tid == 0) L[j][j] = make_double2(s, 0.0);
        for (int i = j + 1 + tid; i < nb; i += 1024) L[i][j] = make_double2(L[i][j].x * inv, L[i][j].y * inv);
    }
    if (fail) {
        if (tid == 0) sc[SC_FLAGS_SLOT] = (double)((int)sc[SC_FLAGS_SLOT] | CRBM_FLAG_CHOLESKY_FAIL);
        return;
    }
    __syncthreads();
    for (int i = ty; i < nb; i += 32)
        for (int j = tx; j <= i; j += 32) A[(k0 + i) * P + k0 + j] = L[i][j];
}

// 2. rows i >= k0 + nb: x L_kk^H = a with x = L_ik, a = A_ik; lane l owns column l of the row.
//    x_m = (a_m - sum_{l<m} x_l conj(L_kk[m][l])) / L_kk[m][m]: once x_l is known (step l, lane l) it is
//    read by every lane, and lanes m > l subtract its term from their own a_m, in the order l = 0, 1, ...
__global__ __launch_bounds__(256) void k_chol_panel(long P, long k0, int nb, double2* __restrict__ A,
                                                    const double* __restrict__ sc) {
    __shared__ double2 L[CH_NB][CH_NB + 1];
    if (chol_failed(sc)) return;
    const int tid = threadIdx.x, lane = tid & 63;
    for (int e = tid; e < nb * nb; e += 256) {
        const int i = e / nb, j = e % nb;
        L[i][j] = (j <= i) ? A[(k0 + i) * P + k0 + j] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    const long i = k0 + nb + (long)blockIdx.x * 4 + (tid >> 6);
    if (i >= P) return;
    double2* row = A + i * P + k0;
    double2 x = lane < nb ? row[lane] : make_double2(0.0, 0.0);
    const double dinv = lane < nb ? 1.0 / L[lane][lane].x : 0.0;   // lane m divides by L_mm at step m
    for (int m = 0; m < nb; ++m) {
        if (lane == m) x = make_double2(x.x * dinv, x.y * dinv);
        const double xr = lane_value(x.x, m), xi = lane_value(x.y, m);
        if (lane > m && lane < nb) {
            const double2 c = L[lane][m];           // x_m conj(L[lane][m])
            x.x -= xr * c.x + xi * c.y;
            x.y -= xi * c.x - xr * c.y;
        }
    }
    if (lane < nb) row[lane] = x;
}

// 3. trailing update of the lower triangle: A_ij -= sum_l L_il conj(L_jl), i >= j >= k1 = k0 + nb.
//    Workgroup = one 32 x 32 tile (I >= J) of the trailing matrix; thread = 2 x 2 outputs.
__global__ __launch_bounds__(256) void k_chol_update(long P, long k0, int nb, double2* __restrict__ A,
                                                     const double* __restrict__ sc) {
    __shared__ double2 Li[CH_T][CH_NB + 1], Lj[CH_T][CH_NB + 1];
    if (chol_failed(sc)) return;
    const long k1 = k0 + nb;
    // tile index -> (I, J), J <= I, over T = ceil((P - k1) / 32) tiles per side
    long rem = blockIdx.x;
    long I = 0;
    while (rem > I) { rem -= I + 1; ++I; }
    const long J = rem;
    const long i0 = k1 + I * CH_T, j0 = k1 + J * CH_T;
    const int tid = threadIdx.x;
    for (int e = tid; e < CH_T * nb; e += 256) {
        const int r = e / nb, l = e % nb;
        Li[r][l] = (i0 + r < P) ? A[(i0 + r) * P + k0 + l] : make_double2(0.0, 0.0);
        Lj[r][l] = (j0 + r < P) ? A[(j0 + r) * P + k0 + l] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    const int ti = (tid >> 4) * 2, tj = (tid & 15) * 2;
    double2 acc[2][2] = {};
    for (int l = 0; l < nb; ++l) {
        const double2 a0 = Li[ti][l], a1 = Li[ti + 1][l], b0 = Lj[tj][l], b1 = Lj[tj + 1][l];
        const double2 a[2] = {a0, a1}, b[2] = {b0, b1};
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                acc[p][q].x += a[p].x * b[q].x + a[p].y * b[q].y;
                acc[p][q].y += a[p].y * b[q].x - a[p].x * b[q].y;
            }
    }
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const long i = i0 + ti + p, j = j0 + tj + q;
            if (i < P && j <= i) {
                double2* dst = A + i * P + j;
                *dst = make_double2(dst->x - acc[p][q].x, dst->y - acc[p][q].y);
            }
        }
}

// L y = F, then L^H x = y, in place in x, by blocks of 64 rows.  Per block: one wave substitutes within
// the diagonal block (each unknown, once known, is read by every lane and the later lanes subtract its
// term), then a kernel over the whole width applies the block's unknowns to the rest: forward, the rows
// below (one wave per row, the lanes over the block's 64 columns); backward, the columns to the left
// (one thread per column, the block's 64 rows in order).

// x = F, or 0 after a failed factorisation
__global__ __launch_bounds__(256) void k_trsv_init(long P, const double2* __restrict__ F, double2* __restrict__ x,
                                                   const double* __restrict__ sc) {
    const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < P) x[k] = chol_failed(sc) ? make_double2(0.0, 0.0) : F[k];
}

// the diagonal block [b0, b0 + nb): forward (L_BB y_B = x_B) or backward (L_BB^H x_B = x_B); four waves
// stage the block, the first substitutes
__global__ __launch_bounds__(256) void k_trsv_diag(long P, const double2* __restrict__ A, long b0, int nb, int backward,
                                                   double2* __restrict__ x, const double* __restrict__ sc) {
    __shared__ double2 D[CH_NB][CH_NB + 1];
    if (chol_failed(sc)) return;
    for (int e = threadIdx.x; e < nb * CH_NB; e += 256) {
        const int r = e / CH_NB, c = e % CH_NB;
        D[r][c] = c <= r ? A[(b0 + r) * P + b0 + c] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    if (threadIdx.x >= 64) return;
    const int lane = threadIdx.x;
    double2 v = lane < nb ? x[b0 + lane] : make_double2(0.0, 0.0);
    const double dinv = lane < nb ? 1.0 / D[lane][lane].x : 0.0;   // lane m divides by L_mm at step m
    if (!backward) {
        // y_m = (x_m - sum_{l<m} L_ml y_l) / L_mm, l = 0, 1, ...
        for (int m = 0; m < nb; ++m) {
            if (lane == m) v = make_double2(v.x * dinv, v.y * dinv);
            const double2 ym = make_double2(lane_value(v.x, m), lane_value(v.y, m));
            if (lane > m && lane < nb) {
                const double2 t = zmul(D[lane][m], ym);
                v.x -= t.x;
                v.y -= t.y;
            }
        }
    } else {
        // x_m = (v_m - sum_{l>m} conj(L_lm) x_l) / L_mm, m from the bottom of the block up
        for (int m = nb - 1; m >= 0; --m) {
            if (lane == m) v = make_double2(v.x * dinv, v.y * dinv);
            const double2 xm = make_double2(lane_value(v.x, m), lane_value(v.y, m));
            if (lane < m) {
                const double2 t = zconjmul(D[m][lane], xm);   // conj(L_m,lane) x_m
                v.x -= t.x;
                v.y -= t.y;
            }
        }
    }
    if (lane < nb) x[b0 + lane] = v;
}

// forward: x_k -= sum_{l < nb} L_k,b0+l y_b0+l for the rows k >= b0 + nb, one wave per row
__global__ __launch_bounds__(256) void k_trsv_rows(long P, const double2* __restrict__ A, long b0, int nb,
                                                   double2* __restrict__ x, const double* __restrict__ sc) {
    if (chol_failed(sc)) return;
    const int lane = threadIdx.x & 63;
    const long k = b0 + nb + (long)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (k >= P) return;
    double2 t = make_double2(0.0, 0.0);
    if (lane < nb) t = zmul(A[k * P + b0 + lane], x[b0 + lane]);
    const double tx = wave_sum(t.x), ty = wave_sum(t.y);
    if (lane == 0) x[k] = make_double2(x[k].x - tx, x[k].y - ty);
}

// backward: x_j -= sum_{r < nb} conj(L_b0+r,j) x_b0+r for the columns j < b0, one thread per column
__global__ __launch_bounds__(256) void k_trsv_cols(long P, const double2* __restrict__ A, long b0, int nb,
                                                   double2* __restrict__ x, const double* __restrict__ sc) {
    if (chol_failed(sc)) return;
    const long j = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= b0) return;
    double ax = 0.0, ay = 0.0;
    for (int r = 0; r < nb; ++r) {
        const double2 t = zconjmul(A[(b0 + r) * P + j], x[b0 + r]);
        ax += t.x;
        ay += t.y;
    }
    x[j] = make_double2(x[j].x - ax, x[j].y - ay);
}

hipError_t launch_cholesky_solve(long P, const float2* S, double eps, const double2* F, double2* A64, double2* x,
                                 double* sc, bool a64_holds_s, hipStream_t stream) {
    if (P < 1 || P > kCholMaxP) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_chol_load, dim3((unsigned)((P * P + 255) / 256)), dim3(256), 0, stream, P,
                       a64_holds_s ? nullptr : S, eps, A64);
    for (long k0 = 0; k0 < P; k0 += CH_NB) {
        const int nb = (int)(P - k0 < CH_NB ? P - k0 : CH_NB);
        hipLaunchKernelGGL(k_chol_diagblock, dim3(1), dim3(1024), 0, stream, P, k0, nb, A64, sc);
        const long rows = P - k0 - nb;
        if (rows <= 0) break;
        hipLaunchKernelGGL(k_chol_panel, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, stream, P, k0, nb, A64, sc);
        const long T = (rows + CH_T - 1) / CH_T;
        hipLaunchKernelGGL(k_chol_update, dim3((unsigned)(T * (T + 1) / 2)), dim3(256), 0, stream, P, k0, nb, A64, sc);
    }
    hipLaunchKernelGGL(k_trsv_init, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, stream, P, F, x, sc);
    const long nblk = (P + CH_NB - 1) / CH_NB;
    for (long blk = 0; blk < nblk; ++blk) {
        const long b0 = blk * CH_NB;
        const int nb = (int)(P - b0 < CH_NB ? P - b0 : CH_NB);
        hipLaunchKernelGGL(k_trsv_diag, dim3(1), dim3(256), 0, stream, P, A64, b0, nb, 0, x, sc);
        const long rows = P - b0 - nb;
        if (rows > 0)
            hipLaunchKernelGGL(k_trsv_rows, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, stream, P, A64, b0, nb, x,
                               sc);
    }
    for (long blk = nblk - 1; blk >= 0; --blk) {
        const long b0 = blk * CH_NB;
        const int nb = (int)(P - b0 < CH_NB ? P - b0 : CH_NB);
        hipLaunchKernelGGL(k_trsv_diag, dim3(1), dim3(256), 0, stream, P, A64, b0, nb, 1, x, sc);
        if (b0 > 0)
            hipLaunchKernelGGL(k_trsv_cols, dim3((unsigned)((b0 + 255) / 256)), dim3(256), 0, stream, P, A64, b0, nb, x,
                               sc);
    }
    return hipGetLastError();
}

}  // namespace crbm
