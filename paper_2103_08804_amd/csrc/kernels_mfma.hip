// Dense S = <O^* O> - <O>^* <O> (Sec. III) on the matrix cores.
//
// The log-derivatives are a Khatri-Rao product: over the extended index
// (i, j), i in [0, N], j in [0, M] (sigma~_N = 1, T~_M = 1),
// O_(i,j)(s) = sigma~_si T~_sj.  A row tile of the output is 4 extended sites
// x 32 extended hidden units, so one workgroup streams only the T values of
// 32 + 32 hidden units and the sign masks of 4 + 4 sites per sample and
// synthesises the 128 + 128 operand rows by XOR-ing the sign into the
// floating-point operands (sigma = +-1 is exact in any format).
//
// Operands are packed K-major (sample index fastest): Tr/Ti planes [Mp][ns]
// and sign masks [Np][ns].  Each workgroup (4 waves) owns a 128 x 128
// complex tile pair (u <= u') and accumulates, per wave, a 64 x 64 complex
// block as 4 real products (RR + II -> Re, RI - IR -> Im) in FP32 with
//   v_mfma_f32_32x32x16_bf16   (BF16 operands), or
//   v_mfma_f32_32x32x2f32      (FP32 operands).
// K tiles of 64 samples are double-buffered through LDS.  The epilogue
// scales by 1/n, subtracts <O_k>^* <O_k'>, maps (i, j) to the parameter
// index and writes the tile and its conjugate transpose.
#include <hip/hip_runtime.h>

#include <vector>

#include "../../include/chebrbm.h"
#include "device.hpp"
#include "internal.hpp"

namespace crbm {

typedef __attribute__((__vector_size__(8 * sizeof(short)))) short bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(int)))) int i32x4;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float floatx16;

constexpr int MK_TI = 4;        // extended sites per row tile
constexpr int MK_TJ = 32;       // extended hidden units per row tile
#ifndef CRBM_MK_KT
#define CRBM_MK_KT 128
#endif
constexpr int MK_KT = CRBM_MK_KT;   // samples per LDS K tile

// ------------------------------------------------------------------ packing
// planes: Tr[jj][s], Ti[jj][s] for jj < Mp (jj == M -> 1 + 0i, jj > M -> 0), s < ns_pad (s >= n -> 0)
// masks:  Sm[ii][s] = sign bit of sigma_si (ii < N), 0 for ii >= N
template <typename E>
__global__ __launch_bounds__(256) void k_pack_t(const float2* __restrict__ T, long n, int M, int Mp, long ns_pad,
                                                E* __restrict__ Tr, E* __restrict__ Ti) {
    __shared__ float2 tile[64][65];
    const long s0 = (long)blockIdx.x * 64;
    const int j0 = blockIdx.y * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int r = ty; r < 64; r += 4) {
        const long s = s0 + r;
        const int j = j0 + tx;
        float2 v = make_float2(0.f, 0.f);
        if (s < n) v = (j < M) ? T[s * M + j] : (j == M ? make_float2(1.f, 0.f) : v);
        tile[r][tx] = v;
    }
    __syncthreads();
    for (int r = ty; r < 64; r += 4) {
        const int j = j0 + r;
        const long s = s0 + tx;
        if (j >= Mp || s >= ns_pad) continue;
        const float2 v = tile[tx][r];
        if constexpr (sizeof(E) == 2) {
            // round to nearest even
            uint32_t ur = __float_as_uint(v.x), ui = __float_as_uint(v.y);
            ur += 0x7FFFu + ((ur >> 16) & 1u);
            ui += 0x7FFFu + ((ui >> 16) & 1u);
            Tr[(long)j * ns_pad + s] = (E)(ur >> 16);
            Ti[(long)j * ns_pad + s] = (E)(ui >> 16);
        } else {
            Tr[(long)j * ns_pad + s] = (E)__float_as_uint(v.x);
            Ti[(long)j * ns_pad + s] = (E)__float_as_uint(v.y);
        }
    }
}

template <typename E>
__global__ __launch_bounds__(256) void k_pack_sig(const int8_t* __restrict__ sig, long n, int N, int Np, long ns_pad,
                                                  E* __restrict__ Sm) {
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)Np * ns_pad) return;
    const int i = (int)(idx / ns_pad);
    const long s = idx % ns_pad;
    E m = 0;
    if (i < N && s < n && sig[s * N + i] < 0) m = (E)(sizeof(E) == 2 ? 0x8000u : 0x80000000u);
    Sm[idx] = m;
}

// ------------------------------------------------------------------ S tiles
__device__ __forceinline__ long ext_to_p(int i, int j, int N, int M) {
    if (i > N || j > M || (i == N && j == M)) return -1;
    if (j == M) return i;
    if (i == N) return (long)N + j;
    return (long)N + M + (long)i * M + j;
}

// Precision policy: BF16 (E = uint16_t, 8 samples per lane fragment) or FP32 (E = uint32_t, 1 sample).
template <bool BF16>
struct Pol;
template <>
struct Pol<true> {
    using E = uint16_t;
    static constexpr int kPerLane = 8;     // K values per lane per MFMA
    static constexpr int kStep = 16;       // samples per MFMA
};
template <>
struct Pol<false> {
    using E = uint32_t;
    static constexpr int kPerLane = 1;
    static constexpr int kStep = 2;
};

template <bool BF16>
__global__ __launch_bounds__(256, 2) void k_sbuild_mfma(int N, int M, long P, int nJ, const int2* __restrict__ order,
                                                        long ns_pad,
                                                        const typename Pol<BF16>::E* __restrict__ Tr,
                                                        const typename Pol<BF16>::E* __restrict__ Ti,
                                                        const typename Pol<BF16>::E* __restrict__ Sm,
                                                        const double2* __restrict__ Om, float inv_n,
                                                        float2* __restrict__ S) {
    using E = typename Pol<BF16>::E;
    constexpr int KT = BF16 ? MK_KT : 64;          // samples per LDS K tile of this precision
    // bytes per LDS row, padded so that the 32 rows of a fragment read fall in distinct banks
    constexpr int ROWB = KT * (int)sizeof(E) + (BF16 ? 16 : 4);
    constexpr int PLANE = MK_TJ * ROWB;                    // one [32][64] plane
    constexpr int MASKS = 2 * MK_TI * ROWB;                // 8 mask rows
    constexpr int STAGE = 4 * PLANE + MASKS;
    __shared__ __attribute__((aligned(16))) unsigned char lds[2 * STAGE];

    // tile pair (u, u'), u <= u', from the dispatch-order table (entries < 0 are padding)
    const int2 pr = order[blockIdx.x];
    if (pr.x < 0) return;
    const long u = pr.x, up = pr.y;
    const int I = (int)(u / nJ), J = (int)(u % nJ);
    const int Ip = (int)(up / nJ), Jp = (int)(up % nJ);

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wi = wave >> 1, wj = wave & 1;

    // global -> LDS assignment: 4 planes of 32 rows x (64 samples) + 8 mask rows
    constexpr int CHUNK = 16;                               // bytes per load
    constexpr int CH_PER_ROW = KT * (int)sizeof(E) / CHUNK;
    const E* plane_src[4] = {Tr + (long)(J * MK_TJ) * ns_pad, Ti + (long)(J * MK_TJ) * ns_pad,
                             Tr + (long)(Jp * MK_TJ) * ns_pad, Ti + (long)(Jp * MK_TJ) * ns_pad};

    floatx16 acc_re[2][2], acc_im[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int v = 0; v < 16; ++v) { acc_re[a][b][v] = 0.f; acc_im[a][b][v] = 0.f; }

    const long n_kt = ns_pad / KT;
    constexpr int PLANE_CHUNKS = MK_TJ * CH_PER_ROW;        // chunks per plane
    constexpr int TOTAL_CHUNKS = 4 * PLANE_CHUNKS + 2 * MK_TI * CH_PER_ROW;
    constexpr int PER_THREAD = (TOTAL_CHUNKS + 255) / 256;
    i32x4 stage_regs[PER_THREAD];

    auto gload = [&](long kt) {
#pragma unroll
        for (int q = 0; q < PER_THREAD; ++q) {
            const int c = tid + q * 256;
            i32x4 v = {0, 0, 0, 0};
            if (c < TOTAL_CHUNKS) {
                const long s_off = kt * KT;
                if (c < 4 * PLANE_CHUNKS) {
                    const int pl = c / PLANE_CHUNKS, rc = c % PLANE_CHUNKS;
                    const int row = rc / CH_PER_ROW, ch = rc % CH_PER_ROW;
                    const E* src = plane_src[pl] + (long)row * ns_pad + s_off + ch * (CHUNK / (int)sizeof(E));
                    v = *reinterpret_cast<const i32x4*>(src);
                } else {
                    const int mc = c - 4 * PLANE_CHUNKS;
                    const int row = mc / CH_PER_ROW, ch = mc % CH_PER_ROW;    // row 0..7
                    const int site = (row < MK_TI) ? I * MK_TI + row : Ip * MK_TI + (row - MK_TI);
                    const E* src = Sm + (long)site * ns_pad + s_off + ch * (CHUNK / (int)sizeof(E));
                    v = *reinterpret_cast<const i32x4*>(src);
                }
            }
            stage_regs[q] = v;
        }
    };
    auto lstore = [&](int buf) {
#pragma unroll
        for (int q = 0; q < PER_THREAD; ++q) {
            const int c = tid + q * 256;
            if (c >= TOTAL_CHUNKS) continue;
            unsigned char* base = lds + buf * STAGE;
            unsigned char* dst;
            if (c < 4 * PLANE_CHUNKS) {
                const int pl = c / PLANE_CHUNKS, rc = c % PLANE_CHUNKS;
                const int row = rc / CH_PER_ROW, ch = rc % CH_PER_ROW;
                dst = base + pl * PLANE + row * ROWB + ch * CHUNK;
            } else {
                const int mc = c - 4 * PLANE_CHUNKS;
                const int row = mc / CH_PER_ROW, ch = mc % CH_PER_ROW;
                dst = base + 4 * PLANE + row * ROWB + ch * CHUNK;
            }
            if constexpr (BF16) {
                *reinterpret_cast<i32x4*>(dst) = stage_regs[q];
            } else {
#pragma unroll
                for (int w4 = 0; w4 < 4; ++w4) reinterpret_cast<int*>(dst)[w4] = stage_regs[q][w4];
            }
        }
    };

    gload(0);
    lstore(0);
    __syncthreads();

    const int lrow = lane & 31, lhalf = lane >> 5;
    for (long kt = 0; kt < n_kt; ++kt) {
        const int buf = (int)(kt & 1);
        if (kt + 1 < n_kt) gload(kt + 1);
        const unsigned char* base = lds + buf * STAGE;
#pragma unroll
        for (int ks = 0; ks < KT; ks += Pol<BF16>::kStep) {
            const int koff = (ks + Pol<BF16>::kPerLane * lhalf) * (int)sizeof(E);
            if constexpr (BF16) {
                const i32x4 trA = *reinterpret_cast<const i32x4*>(base + 0 * PLANE + lrow * ROWB + koff);
                const i32x4 tiA = *reinterpret_cast<const i32x4*>(base + 1 * PLANE + lrow * ROWB + koff);
                const i32x4 trB = *reinterpret_cast<const i32x4*>(base + 2 * PLANE + lrow * ROWB + koff);
                const i32x4 tiB = *reinterpret_cast<const i32x4*>(base + 3 * PLANE + lrow * ROWB + koff);
                i32x4 mA[2], mB[2];
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    mA[a] = *reinterpret_cast<const i32x4*>(base + 4 * PLANE + (2 * wi + a) * ROWB + koff);
                    mB[a] = *reinterpret_cast<const i32x4*>(base + 4 * PLANE + (MK_TI + 2 * wj + a) * ROWB + koff);
                }
                const i32x4 neg = {(int)0x80008000, (int)0x80008000, (int)0x80008000, (int)0x80008000};
                i32x4 ar[2], ai[2], br[2], bi[2], nbr[2];
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    ar[a] = trA ^ mA[a];
                    ai[a] = tiA ^ mA[a];
                    br[a] = trB ^ mB[a];
                    bi[a] = tiB ^ mB[a];
                    nbr[a] = br[a] ^ neg;
                }
                // first product of every accumulator, then the second: eight independent
                // matrix-core operations separate the two updates of one accumulator
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int b = 0; b < 2; ++b) {
                        acc_re[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                            (bf16x8)ar[a], (bf16x8)br[b], acc_re[a][b], 0, 0, 0);
                        acc_im[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                            (bf16x8)ar[a], (bf16x8)bi[b], acc_im[a][b], 0, 0, 0);
                    }
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int b = 0; b < 2; ++b) {
                        acc_re[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                            (bf16x8)ai[a], (bf16x8)bi[b], acc_re[a][b], 0, 0, 0);
                        acc_im[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                            (bf16x8)ai[a], (bf16x8)nbr[b], acc_im[a][b], 0, 0, 0);
                    }
            } else {
                const uint32_t trA = *reinterpret_cast<const uint32_t*>(base + 0 * PLANE + lrow * ROWB + koff);
                const uint32_t tiA = *reinterpret_cast<const uint32_t*>(base + 1 * PLANE + lrow * ROWB + koff);
                const uint32_t trB = *reinterpret_cast<const uint32_t*>(base + 2 * PLANE + lrow * ROWB + koff);
                const uint32_t tiB = *reinterpret_cast<const uint32_t*>(base + 3 * PLANE + lrow * ROWB + koff);
                uint32_t mA[2], mB[2];
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    mA[a] = *reinterpret_cast<const uint32_t*>(base + 4 * PLANE + (2 * wi + a) * ROWB + koff);
                    mB[a] = *reinterpret_cast<const uint32_t*>(base + 4 * PLANE + (MK_TI + 2 * wj + a) * ROWB + koff);
                }
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    const float ar = __uint_as_float(trA ^ mA[a]), ai = __uint_as_float(tiA ^ mA[a]);
#pragma unroll
                    for (int b = 0; b < 2; ++b) {
                        const float br = __uint_as_float(trB ^ mB[b]), bi = __uint_as_float(tiB ^ mB[b]);
                        acc_re[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(ar, br, acc_re[a][b], 0, 0, 0);
                        acc_re[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(ai, bi, acc_re[a][b], 0, 0, 0);
                        acc_im[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(ar, bi, acc_im[a][b], 0, 0, 0);
                        acc_im[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(ai, -br, acc_im[a][b], 0, 0, 0);
                    }
                }
            }
        }
        if (kt + 1 < n_kt) {
            lstore(buf ^ 1);
        }
        __syncthreads();
    }

    // epilogue
    const bool diag = (u == up);
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        const int i = I * MK_TI + 2 * wi + a;
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int ip = Ip * MK_TI + 2 * wj + b;
            const int jp = Jp * MK_TJ + (lane & 31);
            const long kp = ext_to_p(ip, jp, N, M);
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int j = J * MK_TJ + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
                const long k = ext_to_p(i, j, N, M);
                if (k < 0 || kp < 0) continue;
                const double2 ok = Om[k], okp = Om[kp];
                const double2 mm = zconjmul(ok, okp);
                float2 val = make_float2((float)((double)(acc_re[a][b][v] * inv_n) - mm.x),
                                         (float)((double)(acc_im[a][b][v] * inv_n) - mm.y));
                if (k == kp) val.y = 0.f;     // S is Hermitian: its diagonal is real
                S[k * P + kp] = val;
                if (!diag) S[kp * P + k] = cconj(val);
            }
        }
    }
}

// ------------------------------------------------------------------ launcher
hipError_t launch_sbuild_mfma(int N, int M, long P, const int8_t* sig, const float2* T, long n, const double2* Om,
                              float2* S, int prec, void* pack, size_t pack_bytes, const int2* order, long n_order,
                              Profiler* prof, hipStream_t stream) {
    const int Mp = ((M + 1 + MK_TJ - 1) / MK_TJ) * MK_TJ;
    const int Np = ((N + 1 + MK_TI - 1) / MK_TI) * MK_TI;
    const long ns_pad = ((n + MK_KT - 1) / MK_KT) * MK_KT;
    const int nJ = Mp / MK_TJ, nI = Np / MK_TI;
    static_assert(MK_KT % 64 == 0, "the packing grid assumes 64-sample blocks");
    (void)nI;
    const long pairs = n_order;
    const bool bf16 = (prec == CRBM_PREC_BF16);
    const size_t esz = bf16 ? 2 : 4;
    const size_t need = esz * ((size_t)2 * Mp * ns_pad + (size_t)Np * ns_pad);
    if (need > pack_bytes) return hipErrorOutOfMemory;
    const float inv_n = 1.0f / (float)n;
    dim3 gt((unsigned)(ns_pad / 64), (unsigned)((Mp + 63) / 64));
    const long ms = (long)Np * ns_pad;
    if (bf16) {
        uint16_t* Tr = static_cast<uint16_t*>(pack);
        uint16_t* Ti = Tr + (size_t)Mp * ns_pad;
        uint16_t* Sm = Ti + (size_t)Mp * ns_pad;
        prof->begin(PROF_PACK, stream);
        hipLaunchKernelGGL(k_pack_t<uint16_t>, gt, dim3(256), 0, stream, T, n, M, Mp, ns_pad, Tr, Ti);
        hipLaunchKernelGGL(k_pack_sig<uint16_t>, dim3((unsigned)((ms + 255) / 256)), dim3(256), 0, stream, sig, n, N,
                           Np, ns_pad, Sm);
        prof->end(stream);
        prof->begin(PROF_SBUILD, stream);
        hipLaunchKernelGGL(k_sbuild_mfma<true>, dim3((unsigned)pairs), dim3(256), 0, stream, N, M, P, nJ, order,
                           ns_pad, Tr, Ti, Sm, Om, inv_n, S);
        prof->end(stream);
    } else {
        uint32_t* Tr = static_cast<uint32_t*>(pack);
        uint32_t* Ti = Tr + (size_t)Mp * ns_pad;
        uint32_t* Sm = Ti + (size_t)Mp * ns_pad;
        prof->begin(PROF_PACK, stream);
        hipLaunchKernelGGL(k_pack_t<uint32_t>, gt, dim3(256), 0, stream, T, n, M, Mp, ns_pad, Tr, Ti);
        hipLaunchKernelGGL(k_pack_sig<uint32_t>, dim3((unsigned)((ms + 255) / 256)), dim3(256), 0, stream, sig, n, N,
                           Np, ns_pad, Sm);
        prof->end(stream);
        prof->begin(PROF_SBUILD, stream);
        hipLaunchKernelGGL(k_sbuild_mfma<false>, dim3((unsigned)pairs), dim3(256), 0, stream, N, M, P, nJ, order,
                           ns_pad, Tr, Ti, Sm, Om, inv_n, S);
        prof->end(stream);
    }
    return hipGetLastError();
}

// Dispatch order of the tile pairs (u <= u').  Workgroup b runs on XCD b % n_xcd (round-robin
// dispatch), so the pairs are grouped into g x g super-tiles, super-tiles are dealt to the XCDs in
// turn, and each XCD's list is interleaved into the grid: the workgroups one XCD runs together
// then share few operand slabs, which stay in that XCD's L2.  Padding entries are (-1, -1).
std::vector<int2> sbuild_order(int N, int M, int n_xcd, int g) {
    const int Mp = ((M + 1 + MK_TJ - 1) / MK_TJ) * MK_TJ;
    const int Np = ((N + 1 + MK_TI - 1) / MK_TI) * MK_TI;
    const int nt = (Np / MK_TI) * (Mp / MK_TJ);
    const int ns = (nt + g - 1) / g;
    std::vector<std::vector<int2>> per(n_xcd);
    int st = 0;
    for (int U = 0; U < ns; ++U)
        for (int V = U; V < ns; ++V, ++st) {
            std::vector<int2>& L = per[st % n_xcd];
            for (int a = 0; a < g; ++a)
                for (int b = 0; b < g; ++b) {
                    const int u = U * g + a, v = V * g + b;
                    if (u < nt && v < nt && u <= v) L.push_back(make_int2(u, v));
                }
        }
    size_t longest = 0;
    for (auto& L : per) longest = L.size() > longest ? L.size() : longest;
    std::vector<int2> out(longest * n_xcd, make_int2(-1, -1));
    for (int x = 0; x < n_xcd; ++x)
        for (size_t k = 0; k < per[x].size(); ++k) out[k * n_xcd + x] = per[x][k];
    return out;
}

size_t sbuild_pack_bytes(int N, int M, long max_samples) {
    const size_t Mp = ((M + 1 + MK_TJ - 1) / MK_TJ) * MK_TJ;
    const size_t Np = ((N + 1 + MK_TI - 1) / MK_TI) * MK_TI;
    const size_t ns_pad = ((max_samples + MK_KT - 1) / MK_KT) * MK_KT;
    return 4 * (2 * Mp * ns_pad + Np * ns_pad);
}

}  // namespace crbm
