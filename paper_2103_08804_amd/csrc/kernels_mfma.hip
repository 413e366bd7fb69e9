// Dense S = <O^* O> - <O>^* <O> (Sec. III) on the matrix cores.
//
// The log-derivatives are a Khatri-Rao product: with sigma~_N = 1 and the
// extended sites i in [0, N], the W and b parameters are the rows (i, j),
// j in [0, M), with O_(i,j)(s) = sigma~_si T_sj (i = N gives O_b = T), and the
// a parameters are the rows i < N with O_a = sigma_i.
//
// Centring.  Where |<T_j>| is large against the spread of T_j (a unit with
// |Re theta| of a few), raw sums <O^* O> less the product of the means would
// lose the ratio's digits to the operand rounding and to the FP32 sums.  The
// T planes therefore hold T'_j = T_j - c_j with the shift c_j = <T_j> rounded
// to binary32, and the contraction is put back together in double:
//   <O^*_(i,j) O_(i',j')> = <s s' T'^*_j T'_j'> + c_j^* X(i,i',j') + c_j' X(i,i',j)^*
//                           + c_j^* c_j' Y(i,i'),
// X(i,i',j) = <s_i s_i' T'_j>, Y(i,i') = <s_i s_i'> (s = sigma~).  The border
// kernel's sums over a rows are exactly the X and Y with i, i' < N; those with
// an extended site N follow from the means.  The means of the operands the
// contraction sees (T' rounded as packed, plus c) are supplied by the caller,
// so that S stays the centred Gram matrix of one set of vectors.
//
// Main kernel (W and b rows).  A row tile is 8 extended sites x 16 hidden
// units = 128 rows, made of four 32-row matrix-core fragments of 2 sites x 16
// hidden units each; N + 1 sites and M hidden units are padded only to
// multiples of 8 and 16, and the fragments of the last site block that hold
// no real site are skipped (ragged pairs); when that block holds an odd count of
// sites, the half fragment of site N left over in one hidden block is filled
// with site N of the next (a mixed fragment), so that no matrix-core work goes
// to padding.  A workgroup streams, per sample, the T' values of 16 + 16
// hidden units and the sign masks of 8 + 8 sites and synthesises the 128 + 128
// operand rows by XOR-ing the sign bit into the floating-point T' (sigma = +-1
// is exact in any format).  Each workgroup (4 waves) owns a
// 128 x 128 complex tile pair (u <= u') and accumulates, per wave, a 64 x 64
// complex block as 4 real products (RR + II -> Re, RI - IR -> Im) in FP32 with
//   v_mfma_f32_32x32x16_bf16   (BF16 operands), or
//   v_mfma_f32_32x32x2f32      (FP32 operands).
// K tiles of samples are double-buffered through LDS.
//
// Border kernel (a rows).  The a rows are real (sigma_i), so a block of 128 of
// them against a W/b tile needs 2 real products (sigma x sigma' T'_re,
// sigma x sigma' T'_im), and against a block of a rows only one.  Their operand
// is the sign XOR-ed into the sample-weight row (1, or 0 for padded samples).
// It runs first and writes its raw sums (the X and Y above, times n) to an
// N x P side buffer; a last kernel turns them into the a rows and columns of S.
//
// The main epilogue scales by 1/n, adds the shift terms, subtracts
// <O_k>^* <O_k'>, maps the row to the parameter index and writes the block and
// its conjugate transpose.  When the tile pairs are too few to fill the device
// (small P), the sample range is split over `nsplit` workgroups per pair: each
// writes its raw sums to its own slice, and reductions add the slices in split
// order (deterministic, in double) before the same epilogue arithmetic.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <type_traits>
#include <vector>

#include "../../include/chebrbm.h"
#include "device.hpp"
#include "internal.hpp"

namespace crbm {

typedef __attribute__((__vector_size__(8 * sizeof(short)))) short bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(int)))) int i32x4;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float floatx16;

constexpr int MK_TS = 8;        // extended sites per W/b row tile
constexpr int MK_TH = 16;       // hidden units per W/b row tile
constexpr int MK_AB = 128;      // a rows per border block
constexpr int MK_KT = 128;          // sample padding of the packed planes: the largest K tile of any variant
constexpr int MK_KB = 64;           // K tiles per accumulation block (FP32 main kernel: 4096 samples)

struct SbGeom {
    int N, M;
    long P;
    int nSB, nHB;       // site blocks of 8 (over N + 1 extended sites), hidden blocks of 16
    int Np, Mp;         // padded plane heights: 8 nSB mask rows, 16 nHB T rows
};
static SbGeom sb_geom(int N, int M) {
    SbGeom g;
    g.N = N; g.M = M; g.P = (long)N + M + (long)N * M;
    g.nSB = (N + 1 + MK_TS - 1) / MK_TS;
    g.nHB = (M + MK_TH - 1) / MK_TH;
    g.Np = g.nSB * MK_TS;
    g.Mp = g.nHB * MK_TH;
    return g;
}

// ------------------------------------------------------------------ packing
// planes: Tr[j][s], Ti[j][s] = T'_sj = T_sj - c_j for j < Mp (j >= M -> 0), s < ns_pad (s >= n -> 0),
// c_j = shift[N + j] rounded to binary32
// masks:  Sm[i][s] = sign bit of sigma_si (i < N), 0 for i >= N (sigma~_N = 1 and padding);
//         row Np holds the sample weights of the a rows: 1 for s < n, 0 for the padded samples
template <typename E>
__global__ __launch_bounds__(256) void k_pack_t(const float2* __restrict__ T, long n, int N, int M, int Mp,
                                                long ns_pad, const double2* __restrict__ shift,
                                                E* __restrict__ Tr, E* __restrict__ Ti) {
    __shared__ float2 tile[64][65];
    const long s0 = (long)blockIdx.x * 64;
    const int j0 = blockIdx.y * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    float2 c = make_float2(0.f, 0.f);
    if (j0 + tx < M) {
        const double2 cd = shift[N + j0 + tx];
        c = make_float2((float)cd.x, (float)cd.y);
    }
    for (int r = ty; r < 64; r += 4) {
        const long s = s0 + r;
        const int j = j0 + tx;
        float2 v = make_float2(0.f, 0.f);
        if (s < n && j < M) {
            const float2 t = T[s * M + j];
            v = make_float2(t.x - c.x, t.y - c.y);
        }
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
    if (idx >= (long)(Np + 1) * ns_pad) return;
    const int i = (int)(idx / ns_pad);
    const long s = idx % ns_pad;
    E m = 0;
    if (i == Np) m = (s < n) ? (E)(sizeof(E) == 2 ? 0x3F80u : 0x3F800000u) : (E)0;
    else if (i < N && s < n && sig[s * N + i] < 0) m = (E)(sizeof(E) == 2 ? 0x8000u : 0x80000000u);
    Sm[idx] = m;
}

// ------------------------------------------------------------------ parameter index of a row
// W/b row (extended site i, hidden j): W_ij for i < N, b_j for i = N; -1 for padding
__device__ __forceinline__ long wb_to_p(int i, int j, int N, int M) {
    if (i > N || j >= M) return -1;
    if (i == N) return (long)N + j;
    return (long)N + M + (long)i * M + j;
}

// ------------------------------------------------------------------ centring (shift terms in double)
struct Centre {
    const float2* bx;       // [N][P] raw border sums: sum_s sigma_si O'_k(s)  (a rows against every parameter)
    const double2* shift;   // c_j = shift[N + j] rounded to binary32
    const double2* Om;      // <O_k> of the operands as contracted
    double inv_n;
    int N, M;
    long P;
};
__device__ __forceinline__ double2 centre_c(const Centre& c, int j) {
    const double2 v = c.shift[c.N + j];
    return make_double2((double)(float)v.x, (double)(float)v.y);
}
// X(i, i', j) = <s_i s_i' T'_j> for extended sites i, i' in [0, N]; the pair is taken in one order so
// that X is symmetric in (i, i') to the bit
__device__ __forceinline__ double2 centre_x(const Centre& c, int i, int ip, int j) {
    const int lo = i < ip ? i : ip, hi = i < ip ? ip : i;
    if (hi < c.N) {
        const float2 v = c.bx[(long)lo * c.P + (long)c.N + c.M + (long)hi * c.M + j];
        return make_double2((double)v.x * c.inv_n, (double)v.y * c.inv_n);
    }
    const double2 cj = centre_c(c, j);
    if (lo < c.N) {   // <s_i T'_j> = <O_(i,j)> - c_j <sigma_i>
        const double2 w = c.Om[(long)c.N + c.M + (long)lo * c.M + j];
        const double sm = c.Om[lo].x;
        return make_double2(w.x - sm * cj.x, w.y - sm * cj.y);
    }
    const double2 b = c.Om[c.N + j];   // <T'_j> = <O_b_j> - c_j
    return make_double2(b.x - cj.x, b.y - cj.y);
}
// Y(i, i') = <s_i s_i'>: exact integer counts from the border sums, <sigma_i>, or 1
__device__ __forceinline__ double centre_y(const Centre& c, int i, int ip) {
    const int lo = i < ip ? i : ip, hi = i < ip ? ip : i;
    if (hi < c.N) return (double)c.bx[(long)lo * c.P + hi].x * c.inv_n;
    if (lo < c.N) return c.Om[lo].x;
    return 1.0;
}
// S entry of the W/b rows (i, j) = parameter k and (i', j') = parameter kp from
// raw = <s_i s_i' T'^*_j T'_j'>
__device__ __forceinline__ double2 centre_wb(const Centre& c, double2 raw, int i, int j, int ip, int jp, long k,
                                              long kp) {
    const double2 cj = centre_c(c, j), cjp = centre_c(c, jp);
    const double2 x1 = centre_x(c, i, ip, jp), x2 = centre_x(c, i, ip, j);
    const double y = centre_y(c, i, ip);
    double2 v = raw;
    v = zadd(v, zconjmul(cj, x1));                       // c_j^* X(i,i',j')
    v = zadd(v, zconjmul(x2, cjp));                      // X(i,i',j)^* c_j'
    const double2 cc = zconjmul(cj, cjp);
    v = make_double2(v.x + cc.x * y, v.y + cc.y * y);    // c_j^* c_j' Y(i,i')
    return zsub(v, zconjmul(c.Om[k], c.Om[kp]));
}
// extended site and unit of the W/b parameter kp >= N
__device__ __forceinline__ void wb_of_p(long kp, int N, int M, int& i, int& j) {
    if (kp < (long)N + M) { i = N; j = (int)(kp - N); return; }
    const long r = kp - N - M;
    i = (int)(r / M);
    j = (int)(r % M);
}

// Precision policy: BF16 (E = uint16_t, 8 samples per lane fragment) or FP32 (E = uint32_t, 1 sample).
template <bool BF16>
struct Pol;
template <>
struct Pol<true> {
    using E = uint16_t;
    static constexpr int kPerLane = 8;     // K values per lane per MFMA
    static constexpr int kStep = 16;       // samples per MFMA
    static constexpr uint32_t kOne = 0x3F80u;
};
template <>
struct Pol<false> {
    using E = uint32_t;
    static constexpr int kPerLane = 1;
    static constexpr int kStep = 2;
    static constexpr uint32_t kOne = 0x3F800000u;
};

// 16-byte global -> LDS staging of a list of plane rows, through registers
template <int ROWS, int KT, typename E>
struct Stager {
    static constexpr int CHUNK = 16;
    static constexpr int CH_PER_ROW = KT * (int)sizeof(E) / CHUNK;
    static constexpr int TOTAL = ROWS * CH_PER_ROW;
    static constexpr int PER_THREAD = (TOTAL + 255) / 256;
};

// ------------------------------------------------------------------ main kernel: W/b tile pairs
// One tile pair: the A tile (site block sbA, hidden block hbA) against the B tile (sbB, hbB), AF x BF
// fragments per wave.  RAG: A is the last, partly filled site block; every wave takes its first AF
// fragments against fragment `wave` of B.  Else each wave takes 2 x 2 fragments of two full tiles.
// MODE (with RAG), see A_PLAIN: A_MIX when the block holds an odd count of real sites, so that its last
// live fragment holds the extended site N alone and its second half (site N + 1) would be padding; here
// that half is site N of hidden block hbM instead (the b rows of a second hidden block, whose T' rows
// are staged after the masks), so that no matrix-core work goes to padding.  A_DUAL: the fragments of
// two hidden blocks of that block in one workgroup (hbM's T' rows staged after the masks), so that a
// wave issues as many matrix-core operations per operand read as a pair of full tiles.  ROWS_ALLOC: stage rows of the kernel's LDS
// double buffer.  Split mode (nsplit > 1): this workgroup sums the K tiles of split `split` and writes
// raw sums into S + split * P * P (no scaling, no means).
// Helpers of sb_tile_pair, written as functions of their arguments (no closures, so that nothing of a
// tile pair's state has to live in memory when several tile-pair bodies share one kernel).
// The packed-plane row behind stage row `row` (the stage layout of sb_tile_pair).
template <typename E>
__device__ __forceinline__ const E* sb_src_row(int row, const E* Tr, const E* Ti, const E* Sm, long ns_pad, int sbA,
                                               int hbA, int hbM, int sbB, int hbB) {
    if (row < 64 || row >= 80) {
        const int pl = (row < 64 ? row : row - 80) >> 4, r = row & 15;
        const E* plane = (pl & 1) ? Ti : Tr;
        const int hb = row >= 80 ? hbM : (pl < 2) ? hbA : hbB;
        return plane + (long)(hb * MK_TH + r) * ns_pad;
    }
    const int m = row - 64;                      // mask row 0..15
    const int site = (m < MK_TS) ? sbA * MK_TS + m : sbB * MK_TS + (m - MK_TS);
    return Sm + (long)site * ns_pad;
}
// 16-byte chunks tid + 256 q of the stage of K tile kt, global -> registers
template <typename St, int KT, typename E>
__device__ __forceinline__ void sb_gload(i32x4 (&regs)[St::PER_THREAD], long kt, int tid, const E* Tr, const E* Ti,
                                         const E* Sm, long ns_pad, int sbA, int hbA, int hbM, int sbB, int hbB) {
#pragma unroll
    for (int q = 0; q < St::PER_THREAD; ++q) {
        const int c = tid + q * 256;
        i32x4 v = {0, 0, 0, 0};
        if (c < St::TOTAL) {
            const int row = c / St::CH_PER_ROW, ch = c % St::CH_PER_ROW;
            const E* src = sb_src_row<E>(row, Tr, Ti, Sm, ns_pad, sbA, hbA, hbM, sbB, hbB) + kt * KT +
                           ch * (St::CHUNK / (int)sizeof(E));
            v = *reinterpret_cast<const i32x4*>(src);
        }
        regs[q] = v;
    }
}
// the same chunks, registers -> the LDS stage at dst
template <typename St, int ROWB, bool BF16>
__device__ __forceinline__ void sb_lstore(const i32x4 (&regs)[St::PER_THREAD], unsigned char* dst, int tid) {
#pragma unroll
    for (int q = 0; q < St::PER_THREAD; ++q) {
        const int c = tid + q * 256;
        if (c >= St::TOTAL) continue;
        const int row = c / St::CH_PER_ROW, ch = c % St::CH_PER_ROW;
        unsigned char* d = dst + row * ROWB + ch * St::CHUNK;
        if constexpr (BF16) {
            *reinterpret_cast<i32x4*>(d) = regs[q];
        } else {
#pragma unroll
            for (int w4 = 0; w4 < 4; ++w4) reinterpret_cast<int*>(d)[w4] = regs[q][w4];
        }
    }
}
// A-fragment layouts of a tile pair: PLAIN, fragments 0 .. AF-1 of the A tile; MIX, the last of them the
// mixed fragment (site N of hidden blocks hbA and hbM); DUAL, fragments 0 .. AF/2-1 of the last site
// block's tiles of hidden blocks hbA and hbM (the same sites, so the same masks)
constexpr int A_PLAIN = 0, A_MIX = 1, A_DUAL = 2;
// (extended site, hidden unit) of row qq (0..31) of A fragment f
template <int MODE, int AF>
__device__ __forceinline__ int2 sb_row_a(int f, int qq, int N, int sbA, int hbA, int hbM) {
    const int half = qq >> 4;
    if (MODE == A_MIX && f == AF - 1) return make_int2(N, (half ? hbM : hbA) * MK_TH + (qq & 15));
    if (MODE == A_DUAL && f >= AF / 2)
        return make_int2(sbA * MK_TS + 2 * (f - AF / 2) + half, hbM * MK_TH + (qq & 15));
    return make_int2(sbA * MK_TS + 2 * f + half, hbA * MK_TH + (qq & 15));
}

template <bool BF16, int KTB, int AF, int BF, bool RAG, int MODE, int ROWS_ALLOC>
__device__ __forceinline__ void sb_tile_pair(const SbGeom& gm, int sbA, int hbA, int hbM, int sbB, int hbB, bool diag,
                                             int split, long ns_pad, int nsplit,
                                             const typename Pol<BF16>::E* __restrict__ Tr,
                                             const typename Pol<BF16>::E* __restrict__ Ti,
                                             const typename Pol<BF16>::E* __restrict__ Sm, const Centre& cen,
                                             float2* __restrict__ S, unsigned char* lds) {
    using E = typename Pol<BF16>::E;
    constexpr int KT = BF16 ? KTB : 64;            // samples per LDS K tile (BF16: 64 or 128, tuned per plan)
    // bytes per LDS row, padded so that the 16 rows of a fragment read fall in distinct banks
    constexpr int ROWB = KT * (int)sizeof(E) + (BF16 ? 16 : 4);
    // stage rows: [0,16) Tr(A) [16,32) Ti(A) [32,48) Tr(B) [48,64) Ti(B) [64,72) masks(A) [72,80) masks(B);
    // MIX and DUAL: [80,96) Tr(hbM) [96,112) Ti(hbM)
    constexpr int ROWS = MODE != A_PLAIN ? 112 : 80;
    static_assert(ROWS <= ROWS_ALLOC, "the stage rows exceed the LDS buffer");
    static_assert(MODE == A_PLAIN || RAG, "mixed and dual fragments belong to the last site block");
    static_assert(MODE != A_DUAL || AF % 2 == 0, "a dual pair holds as many fragments of each hidden block");
    constexpr int AFH = MODE == A_DUAL ? AF / 2 : AF;   // fragments of hidden block hbA
    constexpr int STAGE = ROWS_ALLOC * ROWB;
    using St = Stager<ROWS, KT, E>;
    const int N = gm.N, M = gm.M;
    const long P = gm.P;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wi = wave >> 1, wj = wave & 1;
    floatx16 acc_re[AF][BF], acc_im[AF][BF];
#pragma unroll
    for (int a = 0; a < AF; ++a)
#pragma unroll
        for (int b = 0; b < BF; ++b)
#pragma unroll
            for (int v = 0; v < 16; ++v) { acc_re[a][b][v] = 0.f; acc_im[a][b][v] = 0.f; }

    i32x4 stage_regs[St::PER_THREAD];
    // this workgroup's K tiles [kt0, kt1): the split ranges are set in 128-sample units, so that every
    // K tile size sums the same samples in the same order
    const long n_kt_all = ns_pad / KT;
    const long per = (ns_pad / MK_KT + nsplit - 1) / nsplit * (MK_KT / KT);
    const long kt0 = split * per < n_kt_all ? split * per : n_kt_all;
    const long kt1 = kt0 + per < n_kt_all ? kt0 + per : n_kt_all;
    if (kt0 < kt1) {
        sb_gload<St, KT, E>(stage_regs, kt0, tid, Tr, Ti, Sm, ns_pad, sbA, hbA, hbM, sbB, hbB);
        sb_lstore<St, ROWB, BF16>(stage_regs, lds, tid);
    }
    __syncthreads();

    const bool raw = nsplit > 1;
    float2* out = S + (raw ? (long)split * P * P : 0L);
    // FP32 operands: the matrix-core accumulators' error grows with the count of accumulations, so the
    // sums run in blocks of MK_KB K tiles (4096 samples), each added to this pair's own entries of the
    // output (its upper tile; FP32 adds on the vector units) and the accumulators cleared
    bool flushed = false;

    // fragment rows: lane row q = lane % 32 is (site 2f + q / 16, hidden q % 16) of fragment f.  The
    // mixed fragment's second half reads the T' rows of hbM (stage row 80 + ...) and has zero masks (site
    // N), so its operands are its rows as they stand; the dual pair's second half reads hbM's rows with
    // the masks of the first half's fragments.
    const int q = lane & 31, lhalf = lane >> 5;
    const int trow = q & 15, qs = q >> 4;
    const int mrow = (MODE == A_MIX && !qs) ? trow : 80 + trow;
    for (long kt = kt0; kt < kt1; ++kt) {
        const int buf = (int)((kt - kt0) & 1);
        if (kt + 1 < kt1) sb_gload<St, KT, E>(stage_regs, kt + 1, tid, Tr, Ti, Sm, ns_pad, sbA, hbA, hbM, sbB, hbB);
        const unsigned char* base = lds + buf * STAGE;
#pragma unroll
        for (int ks = 0; ks < KT; ks += Pol<BF16>::kStep) {
            const int koff = (ks + Pol<BF16>::kPerLane * lhalf) * (int)sizeof(E);
            if constexpr (BF16) {
                const i32x4 trA = *reinterpret_cast<const i32x4*>(base + (0 + trow) * ROWB + koff);
                const i32x4 tiA = *reinterpret_cast<const i32x4*>(base + (16 + trow) * ROWB + koff);
                const i32x4 trB = *reinterpret_cast<const i32x4*>(base + (32 + trow) * ROWB + koff);
                const i32x4 tiB = *reinterpret_cast<const i32x4*>(base + (48 + trow) * ROWB + koff);
                i32x4 trM = trA, tiM = tiA;
                if constexpr (MODE != A_PLAIN) {
                    trM = *reinterpret_cast<const i32x4*>(base + mrow * ROWB + koff);
                    tiM = *reinterpret_cast<const i32x4*>(base + (mrow + 16) * ROWB + koff);
                }
                i32x4 mA[AF], mB[BF];
#pragma unroll
                for (int a = 0; a < AF; ++a) {
                    if (MODE == A_MIX && a == AF - 1) continue;
                    if (a >= AFH) mA[a] = mA[a - AFH];
                    else mA[a] = *reinterpret_cast<const i32x4*>(base + (64 + 2 * (RAG ? a : 2 * wi + a) + qs) * ROWB + koff);
                }
#pragma unroll
                for (int b = 0; b < BF; ++b)
                    mB[b] = *reinterpret_cast<const i32x4*>(base + (72 + 2 * (RAG ? wave : 2 * wj + b) + qs) * ROWB + koff);
                const i32x4 neg = {(int)0x80008000, (int)0x80008000, (int)0x80008000, (int)0x80008000};
                i32x4 ar[AF], ai[AF], br[BF], bi[BF], nbr[BF];
#pragma unroll
                for (int a = 0; a < AF; ++a) {
                    if (MODE == A_MIX && a == AF - 1) {
                        ar[a] = trM;
                        ai[a] = tiM;
                    } else if (a >= AFH) {
                        ar[a] = trM ^ mA[a];
                        ai[a] = tiM ^ mA[a];
                    } else {
                        ar[a] = trA ^ mA[a];
                        ai[a] = tiA ^ mA[a];
                    }
                }
#pragma unroll
                for (int b = 0; b < BF; ++b) {
                    br[b] = trB ^ mB[b];
                    bi[b] = tiB ^ mB[b];
                    nbr[b] = br[b] ^ neg;
                }
                // first product of every accumulator, then the second: independent matrix-core
                // operations separate the two updates of one accumulator
#pragma unroll
                for (int a = 0; a < AF; ++a)
#pragma unroll
                    for (int b = 0; b < BF; ++b) {
                        acc_re[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                            (bf16x8)ar[a], (bf16x8)br[b], acc_re[a][b], 0, 0, 0);
                        acc_im[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                            (bf16x8)ar[a], (bf16x8)bi[b], acc_im[a][b], 0, 0, 0);
                    }
#pragma unroll
                for (int a = 0; a < AF; ++a)
#pragma unroll
                    for (int b = 0; b < BF; ++b) {
                        acc_re[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                            (bf16x8)ai[a], (bf16x8)bi[b], acc_re[a][b], 0, 0, 0);
                        acc_im[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                            (bf16x8)ai[a], (bf16x8)nbr[b], acc_im[a][b], 0, 0, 0);
                    }
            } else {
                const uint32_t trA = *reinterpret_cast<const uint32_t*>(base + (0 + trow) * ROWB + koff);
                const uint32_t tiA = *reinterpret_cast<const uint32_t*>(base + (16 + trow) * ROWB + koff);
                const uint32_t trB = *reinterpret_cast<const uint32_t*>(base + (32 + trow) * ROWB + koff);
                const uint32_t tiB = *reinterpret_cast<const uint32_t*>(base + (48 + trow) * ROWB + koff);
                uint32_t trM = trA, tiM = tiA;
                if constexpr (MODE != A_PLAIN) {
                    trM = *reinterpret_cast<const uint32_t*>(base + mrow * ROWB + koff);
                    tiM = *reinterpret_cast<const uint32_t*>(base + (mrow + 16) * ROWB + koff);
                }
                uint32_t mA[AF], mB[BF];
#pragma unroll
                for (int a = 0; a < AF; ++a)
                    mA[a] = (MODE == A_MIX && a == AF - 1) ? 0u
                            : (a >= AFH) ? mA[a - AFH]
                                         : *reinterpret_cast<const uint32_t*>(
                                               base + (64 + 2 * (RAG ? a : 2 * wi + a) + qs) * ROWB + koff);
#pragma unroll
                for (int b = 0; b < BF; ++b)
                    mB[b] = *reinterpret_cast<const uint32_t*>(base + (72 + 2 * (RAG ? wave : 2 * wj + b) + qs) * ROWB + koff);
#pragma unroll
                for (int a = 0; a < AF; ++a) {
                    const bool second = (MODE == A_MIX && a == AF - 1) || a >= AFH;
                    const uint32_t ra = second ? trM : trA, ia = second ? tiM : tiA;
                    const float ar = __uint_as_float(ra ^ mA[a]), ai = __uint_as_float(ia ^ mA[a]);
#pragma unroll
                    for (int b = 0; b < BF; ++b) {
                        const float br = __uint_as_float(trB ^ mB[b]), bi = __uint_as_float(tiB ^ mB[b]);
                        acc_re[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(ar, br, acc_re[a][b], 0, 0, 0);
                        acc_re[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(ai, bi, acc_re[a][b], 0, 0, 0);
                        acc_im[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(ar, bi, acc_im[a][b], 0, 0, 0);
                        acc_im[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(ai, -br, acc_im[a][b], 0, 0, 0);
                    }
                }
            }
        }
        if (kt + 1 < kt1) sb_lstore<St, ROWB, BF16>(stage_regs, lds + (buf ^ 1) * STAGE, tid);
        if constexpr (!BF16) {
            if ((kt - kt0 + 1) % MK_KB == 0 && kt + 1 < kt1) {
                // an opaque copy of the lane index, so that the entry indices are formed here and not kept
                // live through the K loop
                int ln = lane;
                asm volatile("" : "+v"(ln));
#pragma unroll
                for (int a = 0; a < AF; ++a)
#pragma unroll
                    for (int b = 0; b < BF; ++b) {
                        const int qB = ln & 31, fB = RAG ? wave : 2 * wj + b;
                        const long kp = wb_to_p(sbB * MK_TS + 2 * fB + (qB >> 4), hbB * MK_TH + (qB & 15), N, M);
#pragma unroll
                        for (int v = 0; v < 16; ++v) {
                            const int qA = 8 * (v >> 2) + 4 * (ln >> 5) + (v & 3);
                            const int2 ij = sb_row_a<MODE, AF>(RAG ? a : 2 * wi + a, qA, N, sbA, hbA, hbM);
                            const long k = wb_to_p(ij.x, ij.y, N, M);
                            if (k >= 0 && kp >= 0) {
                                float2* o = out + k * P + kp;
                                const float2 prev = flushed ? *o : make_float2(0.f, 0.f);
                                *o = make_float2(prev.x + acc_re[a][b][v], prev.y + acc_im[a][b][v]);
                            }
                            acc_re[a][b][v] = 0.f;
                            acc_im[a][b][v] = 0.f;
                        }
                    }
                flushed = true;
            }
        }
        __syncthreads();
    }

    // epilogue: accumulator element v of lane l is row 8(v/4) + 4(l/32) + v%4 of the A fragment
    // and column l % 32 of the B fragment
#pragma unroll
    for (int a = 0; a < AF; ++a) {
        const int fA = RAG ? a : 2 * wi + a;
#pragma unroll
        for (int b = 0; b < BF; ++b) {
            const int fB = RAG ? wave : 2 * wj + b;
            const int qB = lane & 31;
            const int iB = sbB * MK_TS + 2 * fB + (qB >> 4), jB = hbB * MK_TH + (qB & 15);
            const long kp = wb_to_p(iB, jB, N, M);
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int qA = 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
                const int2 ij = sb_row_a<MODE, AF>(fA, qA, N, sbA, hbA, hbM);
                const int iA = ij.x, jA = ij.y;
                const long k = wb_to_p(iA, jA, N, M);
                if (k < 0 || kp < 0) continue;
                float2 sum = make_float2(acc_re[a][b][v], acc_im[a][b][v]);
                if (flushed) {
                    const float2 prev = out[k * P + kp];
                    sum = make_float2(prev.x + sum.x, prev.y + sum.y);
                }
                float2 val;
                if (raw) {
                    val = sum;
                } else {
                    const double2 r = make_double2((double)sum.x * cen.inv_n, (double)sum.y * cen.inv_n);
                    const double2 d = centre_wb(cen, r, iA, jA, iB, jB, k, kp);
                    val = make_float2((float)d.x, k == kp ? 0.f : (float)d.y);   // Hermitian: real diagonal
                }
                out[k * P + kp] = val;
                if (!diag) out[kp * P + k] = cconj(val);
            }
        }
    }
}

// Ragged-pair kinds.  The A entry of a ragged pair in the order table holds RAG_FLAG | kind << 26 |
// hM << 13 | h: h (and hM) are hidden blocks of the last site block's tiles, both below 2^13.
constexpr int RAG_PLAIN = 0;   // the first RF fragments of tile h (the last one with its padding half)
constexpr int RAG_MIX = 1;     // the first RF - 1 fragments of tile h, and site N of hidden blocks h and hM
constexpr int RAG_REST = 2;    // the first RF - 1 fragments of tile h (its site N in a RAG_MIX pair)
constexpr int RAG_DUAL = 3;    // the first RF - 1 fragments of tiles h and hM (their sites N in RAG_MIX pairs)
constexpr int RAG_HB_BITS = 13;
constexpr int RAG_FLAG = 1 << 30;
__host__ __device__ constexpr int rag_entry(int kind, int h, int hM) {
    return RAG_FLAG | kind << 26 | hM << RAG_HB_BITS | h;
}
__host__ __device__ constexpr int rag_kind(int x) { return (x >> 26) & 7; }

// The contraction: workgroup x takes tile pair x % n_order of the dispatch-order table (entries < 0 are
// padding): pairs (u, u') of full tiles, u <= u', and, with RF > 0, ragged pairs (rag_entry, u'): the
// last site block's tile of hidden block h (and hM), of whose four 2-site fragments only the first RF
// hold real sites, against tile u'.  One launch takes both, so that the short ragged pairs fill the
// last round of the long ones.
template <bool BF16, int KTB, int RF>
__global__ __launch_bounds__(256, 2) void k_sbuild_mfma(SbGeom gm, const int2* __restrict__ order, long n_order,
                                                        long ns_pad, int nsplit,
                                                        const typename Pol<BF16>::E* __restrict__ Tr,
                                                        const typename Pol<BF16>::E* __restrict__ Ti,
                                                        const typename Pol<BF16>::E* __restrict__ Sm,
                                                        Centre cen, float2* __restrict__ S) {
    using E = typename Pol<BF16>::E;
    constexpr int KT = BF16 ? KTB : 64;
    constexpr int ROWB = KT * (int)sizeof(E) + (BF16 ? 16 : 4);
    constexpr int ROWS_ALLOC = RF ? 112 : 80;
    __shared__ __attribute__((aligned(16))) unsigned char lds[2 * ROWS_ALLOC * ROWB];
    const int split = (int)(blockIdx.x / n_order);
    const int2 pr = order[blockIdx.x % n_order];
    if (pr.x < 0) return;
    const int sbB = pr.y / gm.nHB, hbB = pr.y % gm.nHB;
    if (RF == 0 || !(pr.x & RAG_FLAG)) {
        sb_tile_pair<BF16, KTB, 2, 2, false, A_PLAIN, ROWS_ALLOC>(gm, pr.x / gm.nHB, pr.x % gm.nHB, 0, sbB, hbB,
                                                                pr.x == pr.y, split, ns_pad, nsplit, Tr, Ti, Sm,
                                                                cen, S, lds);
    } else if constexpr (RF > 0) {
        const int kind = rag_kind(pr.x), sbA = gm.nSB - 1;
        const int h = pr.x & ((1 << RAG_HB_BITS) - 1), hM = (pr.x >> RAG_HB_BITS) & ((1 << RAG_HB_BITS) - 1);
        if (kind == RAG_MIX) {
            sb_tile_pair<BF16, KTB, RF, 1, true, A_MIX, ROWS_ALLOC>(gm, sbA, h, hM, sbB, hbB, false, split, ns_pad,
                                                                    nsplit, Tr, Ti, Sm, cen, S, lds);
        } else if (kind == RAG_REST) {
            if constexpr (RF > 1)
                sb_tile_pair<BF16, KTB, RF - 1, 1, true, A_PLAIN, ROWS_ALLOC>(gm, sbA, h, 0, sbB, hbB, false, split,
                                                                              ns_pad, nsplit, Tr, Ti, Sm, cen, S, lds);
        } else if (kind == RAG_DUAL) {
            if constexpr (RF > 1)
                sb_tile_pair<BF16, KTB, 2 * (RF - 1), 1, true, A_DUAL, ROWS_ALLOC>(gm, sbA, h, hM, sbB, hbB, false,
                                                                                   split, ns_pad, nsplit, Tr, Ti, Sm,
                                                                                   cen, S, lds);
        } else {
            sb_tile_pair<BF16, KTB, RF, 1, true, A_PLAIN, ROWS_ALLOC>(gm, sbA, h, 0, sbB, hbB,
                                                                      sbA * gm.nHB + h == pr.y, split, ns_pad,
                                                                      nsplit, Tr, Ti, Sm, cen, S, lds);
        }
    }
}

// ------------------------------------------------------------------ border kernel: a rows
// Workgroup x: a-row block ab = x / nX (rows: sites 128 ab + r) against column set y = x % nX:
// y < nW the W/b tile y, else the a-row block y - nW (blocks with y - nW < ab are skipped).
template <bool BF16>
__global__ __launch_bounds__(256, 2) void k_sbuild_border(SbGeom gm, long ns_pad, int nA, int nsplit,
                                                       const typename Pol<BF16>::E* __restrict__ Tr,
                                                       const typename Pol<BF16>::E* __restrict__ Ti,
                                                       const typename Pol<BF16>::E* __restrict__ Sm,
                                                       float2* __restrict__ bx) {
    using E = typename Pol<BF16>::E;
    constexpr int KT = BF16 ? 64 : 32;
    constexpr int ROWB = KT * (int)sizeof(E) + (BF16 ? 16 : 4);
    // stage rows: [0,128) masks of the a rows; [128,256) the columns: a-row masks, or
    // Tr(16) Ti(16) masks(8) of a W/b tile; 256: the sample weights (1, 0 past n); 257: zeros
    constexpr int ROWS = 258;
    constexpr int STAGE = ROWS * ROWB;
    __shared__ __attribute__((aligned(16))) unsigned char lds[2 * STAGE];
    using St = Stager<ROWS, KT, E>;
    const int nW = gm.nSB * gm.nHB;
    const int nX = nW + nA;
    const int split = (int)(blockIdx.x / (nA * nX));
    const int ab = (blockIdx.x % (nA * nX)) / nX, y = blockIdx.x % nX;
    const bool colA = y >= nW;
    if (colA && y - nW < ab) return;
    const int abB = y - nW;
    const int sbB = colA ? 0 : y / gm.nHB, hbB = colA ? 0 : y % gm.nHB;
    const int N = gm.N, M = gm.M;
    const long P = gm.P;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wi = wave >> 1, wj = wave & 1;
    floatx16 acc_re[2][2], acc_im[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int v = 0; v < 16; ++v) { acc_re[a][b][v] = 0.f; acc_im[a][b][v] = 0.f; }

    i32x4 stage_regs[St::PER_THREAD];
    // source row of stage row `row`, or nullptr for a row of zeros (sites past the mask planes)
    auto src_row = [&](int row) -> const E* {
        if (row == 256) return Sm + (long)gm.Np * ns_pad;
        if (row > 256) return nullptr;
        if (row < 128) {
            const int site = MK_AB * ab + row;
            return site < gm.Np ? Sm + (long)site * ns_pad : nullptr;
        }
        const int r = row - 128;
        if (colA) {
            const int site = MK_AB * abB + r;
            return site < gm.Np ? Sm + (long)site * ns_pad : nullptr;
        }
        if (r < 32) return ((r < 16) ? Tr : Ti) + (long)(hbB * MK_TH + (r & 15)) * ns_pad;
        if (r < 40) return Sm + (long)(sbB * MK_TS + (r - 32)) * ns_pad;
        return nullptr;
    };
    auto gload = [&](long kt) {
#pragma unroll
        for (int qq = 0; qq < St::PER_THREAD; ++qq) {
            const int c = tid + qq * 256;
            i32x4 v = {0, 0, 0, 0};
            if (c < St::TOTAL) {
                const int row = c / St::CH_PER_ROW, ch = c % St::CH_PER_ROW;
                const E* s = src_row(row);
                if (s) v = *reinterpret_cast<const i32x4*>(s + kt * KT + ch * (St::CHUNK / (int)sizeof(E)));
            }
            stage_regs[qq] = v;
        }
    };
    auto lstore = [&](int buf) {
#pragma unroll
        for (int qq = 0; qq < St::PER_THREAD; ++qq) {
            const int c = tid + qq * 256;
            if (c >= St::TOTAL) continue;
            const int row = c / St::CH_PER_ROW, ch = c % St::CH_PER_ROW;
            unsigned char* dst = lds + buf * STAGE + row * ROWB + ch * St::CHUNK;
            if constexpr (BF16) {
                *reinterpret_cast<i32x4*>(dst) = stage_regs[qq];
            } else {
#pragma unroll
                for (int w4 = 0; w4 < 4; ++w4) reinterpret_cast<int*>(dst)[w4] = stage_regs[qq][w4];
            }
        }
    };

    const long n_kt_all = ns_pad / KT;
    const long per = (n_kt_all + nsplit - 1) / nsplit;
    const long kt0 = split * per;
    const long kt1 = kt0 + per < n_kt_all ? kt0 + per : n_kt_all;
    if (kt0 < kt1) {
        gload(kt0);
        lstore(0);
    }
    __syncthreads();
    const int q = lane & 31, lhalf = lane >> 5;
    // per-lane LDS rows of the operands.  A: the a-row masks XOR the sample-weight row.  B: a W/b
    // fragment (T row q % 16, mask row 2 f + q / 16), or a block of a rows (T = the weight row,
    // Ti = the zero row, mask row 32 f + q); so one branch-free pair of products serves both.
    const int rA0 = 32 * (2 * wi + 0) + q, rA1 = 32 * (2 * wi + 1) + q;
    const int rTr = colA ? 256 : 128 + (q & 15);
    const int rTi = colA ? 257 : 144 + (q & 15);
    const int rB0 = colA ? 128 + 32 * (2 * wj + 0) + q : 160 + 2 * (2 * wj + 0) + (q >> 4);
    const int rB1 = colA ? 128 + 32 * (2 * wj + 1) + q : 160 + 2 * (2 * wj + 1) + (q >> 4);
    for (long kt = kt0; kt < kt1; ++kt) {
        const int buf = (int)((kt - kt0) & 1);
        if (kt + 1 < kt1) gload(kt + 1);
        const unsigned char* base = lds + buf * STAGE;
#pragma unroll
        for (int ks = 0; ks < KT; ks += Pol<BF16>::kStep) {
            const int koff = (ks + Pol<BF16>::kPerLane * lhalf) * (int)sizeof(E);
            if constexpr (BF16) {
                const i32x4 wrow = *reinterpret_cast<const i32x4*>(base + 256 * ROWB + koff);
                const i32x4 a_op[2] = {wrow ^ *reinterpret_cast<const i32x4*>(base + rA0 * ROWB + koff),
                                       wrow ^ *reinterpret_cast<const i32x4*>(base + rA1 * ROWB + koff)};
                const i32x4 trB = *reinterpret_cast<const i32x4*>(base + rTr * ROWB + koff);
                const i32x4 tiB = *reinterpret_cast<const i32x4*>(base + rTi * ROWB + koff);
                const i32x4 mB[2] = {*reinterpret_cast<const i32x4*>(base + rB0 * ROWB + koff),
                                     *reinterpret_cast<const i32x4*>(base + rB1 * ROWB + koff)};
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    const i32x4 br = trB ^ mB[b], bi = tiB ^ mB[b];
#pragma unroll
                    for (int a = 0; a < 2; ++a) {
                        acc_re[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16((bf16x8)a_op[a], (bf16x8)br,
                                                                              acc_re[a][b], 0, 0, 0);
                        acc_im[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16((bf16x8)a_op[a], (bf16x8)bi,
                                                                              acc_im[a][b], 0, 0, 0);
                    }
                }
            } else {
                const uint32_t wrow = *reinterpret_cast<const uint32_t*>(base + 256 * ROWB + koff);
                const float a_op[2] = {
                    __uint_as_float(wrow ^ *reinterpret_cast<const uint32_t*>(base + rA0 * ROWB + koff)),
                    __uint_as_float(wrow ^ *reinterpret_cast<const uint32_t*>(base + rA1 * ROWB + koff))};
                const uint32_t trB = *reinterpret_cast<const uint32_t*>(base + rTr * ROWB + koff);
                const uint32_t tiB = *reinterpret_cast<const uint32_t*>(base + rTi * ROWB + koff);
                const uint32_t mB[2] = {*reinterpret_cast<const uint32_t*>(base + rB0 * ROWB + koff),
                                        *reinterpret_cast<const uint32_t*>(base + rB1 * ROWB + koff)};
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    const float br = __uint_as_float(trB ^ mB[b]), bi = __uint_as_float(tiB ^ mB[b]);
#pragma unroll
                    for (int a = 0; a < 2; ++a) {
                        acc_re[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(a_op[a], br, acc_re[a][b], 0, 0, 0);
                        acc_im[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(a_op[a], bi, acc_im[a][b], 0, 0, 0);
                    }
                }
            }
        }
        if (kt + 1 < kt1) lstore(buf ^ 1);
        __syncthreads();
    }

    // epilogue: row = a parameter (site 128 ab + 32 fA + qA); column = W/b row or a parameter.  The raw
    // sums go to row k of the N x P side buffer (of this split's slice); an a-row block writes its
    // transpose as well, so that every entry of the buffer is written.
    const bool diag = colA && abB == ab;
    float2* out = bx + (long)split * N * P;
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        const int fA = 2 * wi + a;
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int fB = 2 * wj + b;
            const int qB = lane & 31;
            long kp;
            if (colA) {
                const int site = MK_AB * abB + 32 * fB + qB;
                kp = site < N ? site : -1;
            } else {
                kp = wb_to_p(sbB * MK_TS + 2 * fB + (qB >> 4), hbB * MK_TH + (qB & 15), N, M);
            }
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int qA = 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
                const int siteA = MK_AB * ab + 32 * fA + qA;
                const long k = siteA < N ? siteA : -1;
                if (k < 0 || kp < 0) continue;
                const float2 val = make_float2(acc_re[a][b][v], acc_im[a][b][v]);
                out[k * P + kp] = val;
                if (colA && !diag) out[kp * P + k] = val;     // Y is real and symmetric
            }
        }
    }
}

// bx = the border sums of the nsplit slices, added in split order in double
__global__ __launch_bounds__(256) void k_bx_reduce(long count, int nsplit, const float2* __restrict__ part,
                                                   float2* __restrict__ bx) {
    const long e = (long)blockIdx.x * 256 + threadIdx.x;
    if (e >= count) return;
    double x = 0.0, y = 0.0;
    for (int s = 0; s < nsplit; ++s) {
        const float2 v = part[(long)s * count + e];
        x += (double)v.x;
        y += (double)v.y;
    }
    bx[e] = make_float2((float)x, (float)y);
}

// The a rows and columns of S from the border sums: k = a_i, kp any parameter,
//   S[a_i][a_i'] = Y(i,i') - <sigma_i><sigma_i'>,
//   S[a_i][(i',j')] = X(i,i',j') + c_j' Y(i,i') - <sigma_i> <O_(i',j')>   (and its conjugate at [kp][k]).
__global__ __launch_bounds__(256) void k_sbuild_arows(Centre cen, float2* __restrict__ S) {
    const long e = (long)blockIdx.x * 256 + threadIdx.x;
    const int N = cen.N, M = cen.M;
    const long P = cen.P;
    if (e >= (long)N * P) return;
    const int i = (int)(e / P);
    const long kp = e % P;
    const double2 mm = zconjmul(cen.Om[i], cen.Om[kp]);
    if (kp < N) {
        const double y = centre_y(cen, i, (int)kp);
        S[(long)i * P + kp] = make_float2((float)(y - mm.x), 0.f);
        return;
    }
    int ip, jp;
    wb_of_p(kp, N, M, ip, jp);
    const double2 x = centre_x(cen, i, ip, jp);
    const double2 cjp = centre_c(cen, jp);
    const double y = centre_y(cen, i, ip);
    const float2 val = make_float2((float)(x.x + cjp.x * y - mm.x), (float)(x.y + cjp.y * y - mm.y));
    S[(long)i * P + kp] = val;
    S[kp * P + i] = cconj(val);
}

// W/b entries of S from the split slices: their sums (in split order, in double) / n with the shift
// terms and the means, real diagonal.  The a rows and columns come from k_sbuild_arows.
__global__ __launch_bounds__(256) void k_sbuild_reduce(Centre cen, int nsplit, const float2* __restrict__ part,
                                                       float2* __restrict__ S) {
    const long P = cen.P;
    const long e = (long)blockIdx.x * 256 + threadIdx.x;
    if (e >= P * P) return;
    const long k = e / P, kp = e % P;
    if (k < cen.N || kp < cen.N) return;
    double x = 0.0, y = 0.0;
    for (int s = 0; s < nsplit; ++s) {
        const float2 v = part[(long)s * P * P + e];
        x += (double)v.x;
        y += (double)v.y;
    }
    int i, j, ip, jp;
    wb_of_p(k, cen.N, cen.M, i, j);
    wb_of_p(kp, cen.N, cen.M, ip, jp);
    const double2 d = centre_wb(cen, make_double2(x * cen.inv_n, y * cen.inv_n), i, j, ip, jp, k, kp);
    S[e] = make_float2((float)d.x, k == kp ? 0.f : (float)d.y);
}

// Live 2-site fragments of the last site block when it holds fewer than seven of the N + 1 extended
// sites (then its tiles go to ragged pairs, which skip the empty fragments), else 0.  For N a multiple
// of 8 the block holds site N alone (one fragment, the b rows); for 10 x 10 it holds sites 96 .. 100.
static int ragged_sites(int N) { return N + 1 - MK_TS * ((N + 1 + MK_TS - 1) / MK_TS - 1); }
int sbuild_ragged_frags(int N) {
    const int f = (ragged_sites(N) + 1) / 2;
    return f < MK_TS / 2 ? f : 0;
}

// The ragged pairs by B tile, with the work of each group in units of one RAG_PLAIN pair
// (live fragments / RF).  When the last block holds an odd count of real sites its last live fragment
// holds site N alone: the tiles of hidden blocks h and h + 1 (h even) then go as one RAG_MIX pair (the
// first RF - 1 fragments of h and the mixed one) and the first RF - 1 fragments of h + 1, which join
// those of the next such h + 3 in one RAG_DUAL pair (an odd one left over as RAG_REST; none when RF = 1):
// 2 RF - 1 fragments where two RAG_PLAIN pairs hold 2 RF.  A last, unpaired hidden block, the pairs
// against the last block's own tiles, and every pair when the count is even, go as RAG_PLAIN.
struct RagGroup {
    std::vector<int2> pairs;
    double work;
};
static std::vector<RagGroup> ragged_groups(int N, int M) {
    std::vector<RagGroup> groups;
    const int rf = sbuild_ragged_frags(N);
    if (!rf) return groups;
    const SbGeom gm = sb_geom(N, M);
    const int nt_main = (gm.nSB - 1) * gm.nHB;
    const bool mix = (ragged_sites(N) & 1) != 0 && gm.nHB < (1 << RAG_HB_BITS);
    const double rest = (double)(rf - 1) / (double)rf;
    for (int up = 0; up < nt_main; ++up) {
        RagGroup g{{}, 0.0};
        std::vector<int> rest_hb;
        int h = 0;
        if (mix) {
            for (; h + 1 < gm.nHB; h += 2) rest_hb.push_back(h + 1);
            if (rf > 1) {
                size_t k = 0;
                for (; k + 1 < rest_hb.size(); k += 2) {
                    g.pairs.push_back(make_int2(rag_entry(RAG_DUAL, rest_hb[k], rest_hb[k + 1]), up));
                    g.work += 2.0 * rest;
                }
                if (k < rest_hb.size()) {
                    g.pairs.push_back(make_int2(rag_entry(RAG_REST, rest_hb[k], 0), up));
                    g.work += rest;
                }
            }
            for (int hm : rest_hb) {
                g.pairs.push_back(make_int2(rag_entry(RAG_MIX, hm - 1, hm), up));
                g.work += 1.0;
            }
        }
        for (; h < gm.nHB; ++h) {
            g.pairs.push_back(make_int2(rag_entry(RAG_PLAIN, h, 0), up));
            g.work += 1.0;
        }
        groups.push_back(g);
    }
    for (int h2 = gm.nHB - 1; h2 >= 0; --h2) {
        RagGroup g{{}, 0.0};
        for (int h = 0; h <= h2; ++h) g.pairs.push_back(make_int2(rag_entry(RAG_PLAIN, h, 0), nt_main + h2));
        g.work = (double)(h2 + 1);
        groups.push_back(g);
    }
    return groups;
}

// Number of sample splits for a contraction of n samples when the tile pairs alone cannot fill the
// device: the split count s (at most max_splits, which the plan's slice buffer holds, and at least 4
// K tiles per split) that minimises the modelled time of the launch,
// ceil(work s / resident workgroups) / s (rounds per unit of one pair's full-sample work; a ragged pair
// of f live fragments counts f / 4), so that the last round of the launch is not left nearly empty.
int sbuild_splits(int N, int M, long n, int n_cu, int max_splits) {
    const SbGeom gm = sb_geom(N, M);
    const int rf = sbuild_ragged_frags(N);
    const long nt = (long)(rf ? gm.nSB - 1 : gm.nSB) * gm.nHB;
    const long n_main = nt * (nt + 1) / 2;
    double w_rag = 0.0;
    for (const RagGroup& g : ragged_groups(N, M)) w_rag += g.work;
    const long n_kt = ((n + MK_KT - 1) / MK_KT * MK_KT) / 64;    // the finest K tile of any variant is 64
    long smax = max_splits < n_kt / 4 ? max_splits : n_kt / 4;
    if (smax < 1) smax = 1;
    const long slots = 2L * n_cu;                                  // two resident workgroups per CU
    double best = 1e300;
    long bs = 1;
    for (long sp = 1; sp <= smax; ++sp) {
        const double w = (double)n_main + 0.25 * rf * w_rag;
        const double t = std::ceil(w * (double)sp / (double)slots - 1e-9) / (double)sp;
        if (t < best * (1.0 - 1e-9)) { best = t; bs = sp; }
    }
    return (int)bs;
}

// Sample splits of the border kernel.  Its nA x (W/b tiles + nA) workgroups each run the whole sample
// range and, for small N, fill few of the resident slots (one K tile in flight per workgroup, so it waits
// on its loads): the split count s (at most max_splits, at least 4 K tiles of 64 per split) that
// minimises ceil(workgroups s / resident workgroups) / s.
int sbuild_border_splits(int N, int M, long n, int n_cu, int max_splits) {
    if (max_splits < 2) return 1;
    const SbGeom gm = sb_geom(N, M);
    const long nA = (N + MK_AB - 1) / MK_AB;
    const long nwg = nA * ((long)gm.nSB * gm.nHB + nA);
    const long n_kt = ((n + MK_KT - 1) / MK_KT * MK_KT) / 64;
    long smax = max_splits < n_kt / 4 ? max_splits : n_kt / 4;
    if (smax < 1) smax = 1;
    const long slots = 2L * n_cu;
    double best = 1e300;
    long bs = 1;
    for (long sp = 1; sp <= smax; ++sp) {
        const double t = (double)((nwg * sp + slots - 1) / slots) / (double)sp;
        if (t < best * (1.0 - 1e-9)) { best = t; bs = sp; }
    }
    return (int)bs;
}

// ------------------------------------------------------------------ launcher
// shift: <O> of the unrounded operands (c_j from its b entries); Om: <O> of the operands as contracted
// (T' rounded as packed, plus c); bx: N x P side buffer; bx_part: nsb of them when the border kernel is
// split nsb > 1 ways over the samples (independently of the nsplit of the tile pairs).
hipError_t launch_sbuild_mfma(int N, int M, long P, const int8_t* sig, const float2* T, long n,
                              const double2* shift, const double2* Om, float2* S, int prec, int kt_bf16, void* pack,
                              size_t pack_bytes, const int2* order, long n_order, float2* split_buf, int nsplit,
                              float2* bx, float2* bx_part, int nsb, Profiler* prof,
                              hipStream_t stream) {
    const SbGeom gm = sb_geom(N, M);
    if (nsplit > 1 && !split_buf) return hipErrorInvalidValue;
    if (nsb < 1 || (nsb > 1 && !bx_part)) return hipErrorInvalidValue;
    if (kt_bf16 != 64 && kt_bf16 != 128) return hipErrorInvalidValue;
    if (!bx) return hipErrorInvalidValue;
    const long ns_pad = ((n + MK_KT - 1) / MK_KT) * MK_KT;
    static_assert(MK_KT % 64 == 0, "the packing grid assumes 64-sample blocks");
    const bool bf16 = (prec == CRBM_PREC_BF16);
    const size_t esz = bf16 ? 2 : 4;
    const size_t need = esz * ((size_t)2 * gm.Mp * ns_pad + (size_t)(gm.Np + 1) * ns_pad);
    if (need > pack_bytes) return hipErrorOutOfMemory;
    Centre cen;
    cen.bx = bx;
    cen.shift = shift;
    cen.Om = Om;
    cen.inv_n = 1.0 / (double)n;
    cen.N = N;
    cen.M = M;
    cen.P = P;
    const dim3 gt((unsigned)(ns_pad / 64), (unsigned)((gm.Mp + 63) / 64));
    const long ms = (long)(gm.Np + 1) * ns_pad;
    const int nA = (N + MK_AB - 1) / MK_AB;
    const int nX = gm.nSB * gm.nHB + nA;
    const long nbx = (long)N * P;
    auto run = [&](auto tag) {
        using E = typename decltype(tag)::E;
        constexpr bool B16 = sizeof(E) == 2;
        E* Tr = static_cast<E*>(pack);
        E* Ti = Tr + (size_t)gm.Mp * ns_pad;
        E* Sm = Ti + (size_t)gm.Mp * ns_pad;
        prof->begin(PROF_PACK, stream);
        hipLaunchKernelGGL(k_pack_t<E>, gt, dim3(256), 0, stream, T, n, N, M, gm.Mp, ns_pad, shift, Tr, Ti);
        hipLaunchKernelGGL(k_pack_sig<E>, dim3((unsigned)((ms + 255) / 256)), dim3(256), 0, stream, sig, n, N, gm.Np,
                           ns_pad, Sm);
        prof->end(stream);
        // the border sums first: the main epilogue reads them
        prof->begin(PROF_SBORDER, stream);
        hipLaunchKernelGGL(k_sbuild_border<B16>, dim3((unsigned)(nA * nX * nsb)), dim3(256), 0, stream, gm, ns_pad,
                           nA, nsb, Tr, Ti, Sm, nsb > 1 ? bx_part : bx);
        if (nsb > 1)
            hipLaunchKernelGGL(k_bx_reduce, dim3((unsigned)((nbx + 255) / 256)), dim3(256), 0, stream, nbx, nsb,
                               bx_part, bx);
        prof->end(stream);
        prof->begin(PROF_SBUILD, stream);
        float2* out = nsplit > 1 ? split_buf : S;
        const dim3 grid((unsigned)(n_order * nsplit));
        // the FP32 variant has one K tile (64) whatever kt_bf16 says
        auto launch = [&](auto rf_tag, const int2* ord, long n_ord) {
            constexpr int R = decltype(rf_tag)::value;
            const dim3 g((unsigned)(n_ord * nsplit));
            if (B16 && kt_bf16 == 64)
                hipLaunchKernelGGL((k_sbuild_mfma<B16, 64, R>), g, dim3(256), 0, stream, gm, ord, n_ord, ns_pad,
                                   nsplit, Tr, Ti, Sm, cen, out);
            else
                hipLaunchKernelGGL((k_sbuild_mfma<B16, 128, R>), g, dim3(256), 0, stream, gm, ord, n_ord, ns_pad,
                                   nsplit, Tr, Ti, Sm, cen, out);
        };
        switch (sbuild_ragged_frags(N)) {
            case 1: launch(std::integral_constant<int, 1>{}, order, n_order); break;
            case 2: launch(std::integral_constant<int, 2>{}, order, n_order); break;
            case 3: launch(std::integral_constant<int, 3>{}, order, n_order); break;
            default: launch(std::integral_constant<int, 0>{}, order, n_order); break;
        }
        prof->end(stream);
        prof->begin(PROF_SBORDER, stream);
        if (nsplit > 1)
            hipLaunchKernelGGL(k_sbuild_reduce, dim3((unsigned)((P * P + 255) / 256)), dim3(256), 0, stream, cen,
                               nsplit, split_buf, S);
        hipLaunchKernelGGL(k_sbuild_arows, dim3((unsigned)((nbx + 255) / 256)), dim3(256), 0, stream, cen, S);
        prof->end(stream);
    };
    if (bf16) run(Pol<true>{});
    else run(Pol<false>{});
    return hipGetLastError();
}

// Dispatch order of the W/b tile pairs (u <= u').  Workgroup b runs on XCD b % n_xcd (round-robin
// dispatch), so the pairs are grouped into g x g super-tiles, super-tiles are dealt to the XCDs in
// turn, and each XCD's list is interleaved into the grid: the workgroups one XCD runs together
// then share few operand slabs, which stay in that XCD's L2.  Padding entries are (-1, -1).
std::vector<int2> sbuild_order(int N, int M, int n_xcd, int g) {
    const SbGeom gm = sb_geom(N, M);
    // with ragged pairs the main kernel takes the tiles of the full site blocks only
    const int nt = (sbuild_ragged_frags(N) ? gm.nSB - 1 : gm.nSB) * gm.nHB;
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

// Ragged pairs in dispatch order, after the pairs of full tiles: kind by kind, the longest first
// (RAG_DUAL, then RAG_MIX and RAG_PLAIN, then RAG_REST), each kind by B tile.  Workgroups of one kind then
// run side by side and the shortest fill the last round.
std::vector<int2> sbuild_order_ragged(int N, int M) {
    std::vector<int2> out;
    const std::vector<RagGroup> groups = ragged_groups(N, M);
    const int kinds[] = {RAG_DUAL, RAG_MIX, RAG_PLAIN, RAG_REST};
    for (int kind : kinds)
        for (const RagGroup& g : groups)
            for (const int2& e : g.pairs)
                if (rag_kind(e.x) == kind) out.push_back(e);
    return out;
}

size_t sbuild_pack_bytes(int N, int M, long max_samples) {
    const SbGeom gm = sb_geom(N, M);
    const size_t ns_pad = ((max_samples + MK_KT - 1) / MK_KT) * MK_KT;
    return 4 * (2 * (size_t)gm.Mp * ns_pad + (size_t)(gm.Np + 1) * ns_pad);
}

}  // namespace crbm
