// Ceiling probes for the rooflines: the sustained rate of the BF16 matrix cores and of HBM on the
// device at hand, next to the datasheet figures.
//
// Matrix cores: every wave keeps eight independent 32x32x16 BF16 accumulators and issues nothing
// but matrix-core operations in its loop (operands stay in registers, non-zero data).
// HBM: a grid-stride 16-byte copy between two buffers far larger than the caches.
#include <hip/hip_runtime.h>

#include "device.hpp"


namespace crbm {

typedef __attribute__((__vector_size__(8 * sizeof(short)))) short pbf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float pfloatx16;

__global__ __launch_bounds__(256) void k_probe_mfma(int iters, float* __restrict__ out) {
    const int t = threadIdx.x;
    // small non-zero BF16 operands from an integer hash of the lane (no memory reads)
    pbf16x8 op[4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            uint32_t h = (uint32_t)(t * 8 + e + 977 * q) * 2654435761u;
            h ^= h >> 15;
            const float f = ((float)(h >> 8) * (1.0f / 16777216.0f) - 0.5f) * 0.02f;
            op[q][e] = (short)(__float_as_uint(f) >> 16);
        }
    pfloatx16 acc[8];
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[i][v] = 0.f;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int i = 0; i < 8; ++i)
            acc[i] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(op[i & 3], op[(i >> 2) + 2 * (i & 1)], acc[i], 0, 0, 0);
    }
    float s = 0.f;
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int v = 0; v < 16; ++v) s += acc[i][v];
    out[(long)blockIdx.x * 256 + t] = s;
}

__global__ __launch_bounds__(256) void k_probe_copy(const int4* __restrict__ src, int4* __restrict__ dst, long n) {
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256) dst[i] = src[i];
}

// Re log(2 cosh z) in the Metropolis sweep's form (hardware exp, cos, log), eight independent chains
// per lane, one add per evaluation and no memory traffic.
__global__ __launch_bounds__(256) void k_probe_logcosh(int iters, float* __restrict__ out) {
    const int t = blockIdx.x * 256 + threadIdx.x;
    float2 z[8];
    float acc[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        z[i] = make_float2(0.01f * (float)(t % 97) + 0.1f * (float)i, 0.02f * (float)(t % 89) - 0.05f * (float)i);
        acc[i] = 0.f;
    }
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            acc[i] += re_log2cosh_fast(z[i]);
            z[i].x += 1e-4f;
        }
    }
    float s = 0.f;
#pragma unroll
    for (int i = 0; i < 8; ++i) s += acc[i];
    out[t] = s;
}

// Whole-row reads of a small complex64 table (n_rows x M, L2-resident) at pseudo-random rows, lanes over
// the row: the Metropolis sweep's W-row gathers.
__global__ __launch_bounds__(256) void k_probe_gather(const float2* __restrict__ tab, int n_rows, int M, int iters,
                                                      float* __restrict__ out) {
    const int lane = threadIdx.x & 63;
    const unsigned wave = blockIdx.x * 4 + (threadIdx.x >> 6);
    float acc = 0.f;
    for (int it = 0; it < iters; ++it) {
        uint32_t h = (wave * 2654435761u) ^ ((uint32_t)it * 40503u);
        h ^= h >> 13;
        h *= 0x5bd1e995u;
        h ^= h >> 15;
        const int row = (int)(h % (uint32_t)n_rows);
        for (int k = lane; k < M; k += 64) {
            const float2 v = tab[(long)row * M + k];
            acc += v.x + v.y;
        }
    }
    out[blockIdx.x * 256 + threadIdx.x] = acc;
}

hipError_t launch_probe_logcosh(int blocks, int iters, float* out, hipStream_t stream) {
    hipLaunchKernelGGL(k_probe_logcosh, dim3(blocks), dim3(256), 0, stream, iters, out);
    return hipGetLastError();
}
hipError_t launch_probe_gather(int blocks, const void* tab, int n_rows, int M, int iters, float* out,
                               hipStream_t stream) {
    hipLaunchKernelGGL(k_probe_gather, dim3(blocks), dim3(256), 0, stream, static_cast<const float2*>(tab), n_rows,
                       M, iters, out);
    return hipGetLastError();
}
hipError_t launch_probe_mfma(int blocks, int iters, float* out, hipStream_t stream) {
    hipLaunchKernelGGL(k_probe_mfma, dim3(blocks), dim3(256), 0, stream, iters, out);
    return hipGetLastError();
}

hipError_t launch_probe_copy(int blocks, const void* src, void* dst, long n16, hipStream_t stream) {
    hipLaunchKernelGGL(k_probe_copy, dim3(blocks), dim3(256), 0, stream, static_cast<const int4*>(src),
                       static_cast<int4*>(dst), n16);
    return hipGetLastError();
}

}  // namespace crbm
