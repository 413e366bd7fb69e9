// Dense Hermitian positive-definite solve (S + eps I) x = F in double precision
// by a left-looking Cholesky factorisation L L^H followed by two triangular
// solves.  Used for the natural-gradient system of Sec. III when P is a few
// thousand (the factorisation costs P^3/3 complex multiply-adds).
#include "../../include/chebrbm.h"
#include "device.hpp"
#include "internal.hpp"

namespace crbm {

enum { SC_FLAGS_SLOT = 15 };   // must match the scalar layout of the step driver
constexpr long kCholMaxP = 4000;  // the triangular solves keep x in LDS (16 B per entry, < 64 KB)

// A64 = S + eps I (lower triangle used)
__global__ __launch_bounds__(256) void k_chol_load(long P, const float2* __restrict__ S, double eps,
                                                   double2* __restrict__ A) {
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= P * P) return;
    const long i = idx / P, j = idx % P;
    const float2 v = S[idx];
    A[idx] = make_double2((double)v.x + (i == j ? eps : 0.0), (double)v.y);
}

// diagonal of column j: L_jj = sqrt(A_jj - sum_{k<j} |L_jk|^2)   (one wave)
__global__ __launch_bounds__(64) void k_chol_diag(long P, long j, double2* __restrict__ A, double* __restrict__ sc) {
    if ((int)sc[SC_FLAGS_SLOT] & CRBM_FLAG_CHOLESKY_FAIL) return;
    const int lane = threadIdx.x;
    const double2* row = A + j * P;
    double acc = 0.0;
    for (long k = lane; k < j; k += 64) acc += row[k].x * row[k].x + row[k].y * row[k].y;
    acc = wave_sum(acc);
    if (lane == 0) {
        const double d = A[j * P + j].x - acc;
        if (!(d > 0.0) || !isfinite(d)) {
            sc[SC_FLAGS_SLOT] = (double)((int)sc[SC_FLAGS_SLOT] | CRBM_FLAG_CHOLESKY_FAIL);
            return;
        }
        A[j * P + j] = make_double2(sqrt(d), 0.0);
    }
}

// rows i > j: L_ij = (A_ij - sum_{k<j} L_ik conj(L_jk)) / L_jj   (one wave per row)
__global__ __launch_bounds__(256) void k_chol_col(long P, long j, double2* __restrict__ A, const double* __restrict__ sc) {
    if ((int)sc[SC_FLAGS_SLOT] & CRBM_FLAG_CHOLESKY_FAIL) return;
    const int lane = threadIdx.x & 63;
    const long i = j + 1 + (long)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= P) return;
    const double2* ri = A + i * P;
    const double2* rj = A + j * P;
    double ax = 0.0, ay = 0.0;
    for (long k = lane; k < j; k += 64) {
        const double2 t = zmul(ri[k], make_double2(rj[k].x, -rj[k].y));
        ax += t.x;
        ay += t.y;
    }
    ax = wave_sum(ax);
    ay = wave_sum(ay);
    if (lane == 0) {
        const double ljj = A[j * P + j].x;
        A[i * P + j] = make_double2((A[i * P + j].x - ax) / ljj, (A[i * P + j].y - ay) / ljj);
    }
}

// L y = F, then L^H x = y; one block, rows in sequence, each dot product split over the block
__global__ __launch_bounds__(1024) void k_chol_solve(long P, const double2* __restrict__ A,
                                                     const double2* __restrict__ F, double2* __restrict__ xg,
                                                     const double* __restrict__ sc) {
    __shared__ double shx[16], shy[16];
    extern __shared__ double2 x[];                 // the solution lives in LDS (P <= kCholMaxP)
    const bool failed = ((int)sc[SC_FLAGS_SLOT] & CRBM_FLAG_CHOLESKY_FAIL) != 0;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    if (failed) {
        for (long k = tid; k < P; k += blockDim.x) xg[k] = make_double2(0.0, 0.0);
        return;
    }
    for (long i = 0; i < P; ++i) {                 // forward: y_i = (F_i - sum_{k<i} L_ik y_k) / L_ii
        double ax = 0.0, ay = 0.0;
        for (long k = tid; k < i; k += blockDim.x) {
            const double2 t = zmul(A[i * P + k], x[k]);
            ax += t.x;
            ay += t.y;
        }
        ax = wave_sum(ax);
        ay = wave_sum(ay);
        if (lane == 0) { shx[wv] = ax; shy[wv] = ay; }
        __syncthreads();
        if (tid == 0) {
            double sx = 0.0, sy = 0.0;
            for (int w = 0; w < (int)(blockDim.x >> 6); ++w) { sx += shx[w]; sy += shy[w]; }
            const double lii = A[i * P + i].x;
            x[i] = make_double2((F[i].x - sx) / lii, (F[i].y - sy) / lii);
        }
        __syncthreads();
    }
    for (long i = P - 1; i >= 0; --i) {            // backward: x_i = (y_i - sum_{k>i} conj(L_ki) x_k) / L_ii
        double ax = 0.0, ay = 0.0;
        for (long k = i + 1 + tid; k < P; k += blockDim.x) {
            const double2 t = zconjmul(A[k * P + i], x[k]);
            ax += t.x;
            ay += t.y;
        }
        ax = wave_sum(ax);
        ay = wave_sum(ay);
        if (lane == 0) { shx[wv] = ax; shy[wv] = ay; }
        __syncthreads();
        if (tid == 0) {
            double sx = 0.0, sy = 0.0;
            for (int w = 0; w < (int)(blockDim.x >> 6); ++w) { sx += shx[w]; sy += shy[w]; }
            const double lii = A[i * P + i].x;
            x[i] = make_double2((x[i].x - sx) / lii, (x[i].y - sy) / lii);
        }
        __syncthreads();
    }
    for (long k = tid; k < P; k += blockDim.x) xg[k] = x[k];
}

hipError_t launch_cholesky_solve(long P, const float2* S, double eps, const double2* F, double2* A64, double2* x,
                                 double* sc, hipStream_t stream) {
    hipLaunchKernelGGL(k_chol_load, dim3((unsigned)((P * P + 255) / 256)), dim3(256), 0, stream, P, S, eps, A64);
    for (long j = 0; j < P; ++j) {
        hipLaunchKernelGGL(k_chol_diag, dim3(1), dim3(64), 0, stream, P, j, A64, sc);
        const long rows = P - j - 1;
        if (rows > 0)
            hipLaunchKernelGGL(k_chol_col, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, stream, P, j, A64, sc);
    }
    hipLaunchKernelGGL(k_chol_solve, dim3(1), dim3(1024), (size_t)P * sizeof(double2), stream, P, A64, F, x, sc);
    return hipGetLastError();
}

}  // namespace crbm
