// Device-side building blocks shared by the gfx950 kernels: complex float
// arithmetic, the Philox4x32-10 counter-based generator, log(2 cosh z) and
// tanh z for complex z, and wave64 reductions.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace crbm {

constexpr int kWave = 64;

// ---------------------------------------------------------------- complex float
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float2 cdiv(float2 a, float2 b) {
    // Smith's algorithm keeps the intermediate magnitudes bounded
    if (fabsf(b.x) >= fabsf(b.y)) {
        float r = b.y / b.x, d = b.x + b.y * r;
        return make_float2((a.x + a.y * r) / d, (a.y - a.x * r) / d);
    }
    float r = b.x / b.y, d = b.x * r + b.y;
    return make_float2((a.x * r + a.y) / d, (a.y * r - a.x) / d);
}
__device__ __forceinline__ float2 cexpf(float2 z) {
    float e = expf(z.x), s, c;
    sincosf(z.y, &s, &c);
    return make_float2(e * c, e * s);
}

// (cos x, sin x) of a float: x = k pi/2 + r by the Cody-Waite reduction (pi/2 = P1 + P2 + P3, each
// k Pi removed by one fused multiply-add), r in [-pi/4, pi/4], then the Taylor series of sin r to r^9
// and of cos r to r^10 (truncation below 2e-9) and the quadrant k mod 4.  About one ulp for
// |x| < 3000.  The library sincos carries a large-argument reduction whose code and registers every
// kernel that evaluates log cosh per hidden unit would pay for.
__device__ __forceinline__ float2 cos_sin(float x) {
    const float k = rintf(x * 0.63661977f);
    float r = fmaf(-k, 1.5703125f, x);
    r = fmaf(-k, 4.837512969970703e-4f, r);
    r = fmaf(-k, 7.549790126404332e-8f, r);
    const float r2 = r * r;
    float ps = fmaf(r2, 2.7557319e-6f, -1.9841270e-4f);
    ps = fmaf(r2, ps, 8.3333338e-3f);
    ps = fmaf(r2, ps, -0.16666667f);
    ps = fmaf(r2, ps, 1.f);
    const float sr = r * ps;
    float pc = fmaf(r2, -2.7557320e-7f, 2.4801588e-5f);
    pc = fmaf(r2, pc, -1.3888889e-3f);
    pc = fmaf(r2, pc, 4.1666668e-2f);
    pc = fmaf(r2, pc, -0.5f);
    const float cr = fmaf(r2, pc, 1.f);
    const int q = (int)k & 3;
    const float c = (q == 0) ? cr : (q == 1) ? -sr : (q == 2) ? -cr : sr;
    const float sn = (q == 0) ? sr : (q == 1) ? cr : (q == 2) ? -sr : -cr;
    return make_float2(c, sn);
}

// log 2cosh z = s z + log 2 + log f, f = (1 + e^{-2 s z}) / 2, s = sign Re z, |f| <= 1: adds s z to lin
// and multiplies f into p
__device__ __forceinline__ void cosh_factor(float2 z, float sign, float2& lin, float2& p) {
    const float sg = z.x >= 0.f ? 1.f : -1.f;
    const float ex = expf(-2.f * fabsf(z.x));
    const float2 cs = cos_sin(2.f * sg * z.y);
    lin.x += sign * fabsf(z.x);
    lin.y += sign * sg * z.y;
    p = cmul(p, make_float2(0.5f * (1.f + ex * cs.x), -0.5f * ex * cs.y));
}

// double complex
__device__ __forceinline__ double2 zadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 zsub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 zmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 zconjmul(double2 a, double2 b) {  // conj(a) * b
    return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ double2 zdiv(double2 a, double2 b) {
    double d = b.x * b.x + b.y * b.y;
    return make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}

// ---------------------------------------------------------------- Philox4x32-10
// Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3"
// (SC'11): ten rounds of the 4x32 bijection, round keys advanced by the Weyl
// increments.  Counter (c0, c1, c2, c3), key (k0, k1).
struct u32x4 { uint32_t x, y, z, w; };

__device__ __forceinline__ u32x4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                uint32_t k0, uint32_t k1) {
    constexpr uint32_t kMulA = 0xD2511F53u, kMulB = 0xCD9E8D57u;
    constexpr uint32_t kWeylA = 0x9E3779B9u, kWeylB = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t hiA = __umulhi(kMulA, c0), loA = kMulA * c0;
        const uint32_t hiB = __umulhi(kMulB, c2), loB = kMulB * c2;
        const uint32_t n0 = hiB ^ c1 ^ k0, n2 = hiA ^ c3 ^ k1;
        c0 = n0; c1 = loB; c2 = n2; c3 = loA;
        k0 += kWeylA; k1 += kWeylB;
    }
    return {c0, c1, c2, c3};
}

// Stream layout used throughout: key = (seed lo, seed hi), counter = (a, b lo, b hi, tag).
__device__ __forceinline__ u32x4 draw(uint64_t seed, uint32_t a, uint64_t b, uint32_t tag) {
    return philox4x32_10(a, (uint32_t)b, (uint32_t)(b >> 32), tag, (uint32_t)seed, (uint32_t)(seed >> 32));
}
__device__ __forceinline__ int draw_index(uint32_t x, int n) { return (int)__umulhi(x, (uint32_t)n); }
__device__ __forceinline__ float draw_unit(uint32_t x) { return (float)(x >> 8) * (1.0f / 16777216.0f); }

// ---------------------------------------------------------------- near the zeros of cosh
// cosh z vanishes at z = i pi (m + 1/2), where complex RBMs put hidden units to represent nodes of a
// state.  A binary32 theta locates such a zero only to its own rounding (about 1e-7 |theta| after the sum
// over sites), so cosh, tanh and log cosh at distance d from it carry relative errors near 1e-7 / d.  A
// unit whose binary32 theta lies within kPoleBand of a zero (in both parts) is therefore re-evaluated:
// theta in double from the sample's spins and the parameters (each term is a binary32 value, so the sum is
// exact while the terms span fewer than about 25 binary orders of magnitude), delta = theta - i pi (m + 1/2)
// with pi to about 32 digits, and
//   cosh theta = i (-1)^m sinh delta,  log cosh theta = log sinh delta + i pi (m + 1/2),  tanh theta = coth delta.
constexpr float kPoleBand = 0.5f;
constexpr double kPiLo = 1.2246467991473532e-16;   // pi minus the double nearest pi

__device__ __forceinline__ bool near_pole(float2 z) {
    if (!(fabsf(z.x) < kPoleBand)) return false;
    const float m = rintf(fmaf(z.y, 0.31830988618379067f, -0.5f));
    return fabsf(fmaf(-3.14159265358979f, m + 0.5f, z.y)) < kPoleBand;
}

// theta_k = b_k + sum_i s_i W_ik in double over one sample's spins
__device__ __forceinline__ double2 theta_double(const int8_t* __restrict__ srow, int N, int M, int k,
                                                const float2* __restrict__ b, const float2* __restrict__ W) {
    double x = (double)b[k].x, y = (double)b[k].y;
    for (int i = 0; i < N; ++i) {
        const float2 w = W[(long)i * M + k];
        const double s = (double)srow[i];
        x = fma(s, (double)w.x, x);
        y = fma(s, (double)w.y, y);
    }
    return make_double2(x, y);
}

// delta = t - i pi (m + 1/2) for the zero of cosh nearest to t (pi to about 32 digits); h = m + 1/2
__device__ __forceinline__ double2 pole_offset(double2 t, double& h) {
    const double m = rint(t.y * 0.31830988618379067 - 0.5);
    h = m + 0.5;
    const double hi = 3.141592653589793 * h, err = fma(3.141592653589793, h, -hi);
    return make_double2(t.x, ((t.y - hi) - err) - kPiLo * h);
}

// sinh d and cosh d of a complex d with |Re d|, |Im d| < 0.6, by the Taylor series of sinh, cosh, sin and cos
// (truncation below 1e-19 relative)
__device__ __forceinline__ void sinh_cosh_small(double2 d, double2& sh, double2& ch) {
    const double dx = d.x, dy = d.y, x2 = dx * dx, y2 = dy * dy;
    const double shx = dx * (1.0 + x2 / 6.0 * (1.0 + x2 / 20.0 * (1.0 + x2 / 42.0 * (1.0 + x2 / 72.0 * (1.0 + x2 / 110.0 *
                       (1.0 + x2 / 156.0 * (1.0 + x2 / 210.0)))))));
    const double chx = 1.0 + x2 / 2.0 * (1.0 + x2 / 12.0 * (1.0 + x2 / 30.0 * (1.0 + x2 / 56.0 * (1.0 + x2 / 90.0 *
                       (1.0 + x2 / 132.0 * (1.0 + x2 / 182.0 * (1.0 + x2 / 240.0)))))));
    const double sy = dy * (1.0 - y2 / 6.0 * (1.0 - y2 / 20.0 * (1.0 - y2 / 42.0 * (1.0 - y2 / 72.0 * (1.0 - y2 / 110.0 *
                      (1.0 - y2 / 156.0 * (1.0 - y2 / 210.0)))))));
    const double cy = 1.0 - y2 / 2.0 * (1.0 - y2 / 12.0 * (1.0 - y2 / 30.0 * (1.0 - y2 / 56.0 * (1.0 - y2 / 90.0 *
                      (1.0 - y2 / 132.0 * (1.0 - y2 / 182.0 * (1.0 - y2 / 240.0)))))));
    sh = make_double2(shx * cy, chx * sy);
    ch = make_double2(chx * cy, shx * sy);
}

// log cosh theta (without log 2) and tanh theta, rounded to binary32, from theta in double near a zero of
// cosh; the logarithm of the modulus on a power-of-two scaled copy, so that a modulus below the binary32
// range still has its logarithm.
__device__ __forceinline__ void pole_eval(double2 t, float2& lc, float2& th) {
    double h;
    double2 sh, ch;
    sinh_cosh_small(pole_offset(t, h), sh, ch);
    const int e = ilogb(fmax(fabs(sh.x), fabs(sh.y)));
    const float ur = (float)ldexp(sh.x, -e), ui = (float)ldexp(sh.y, -e);
    constexpr float kLn2 = 0.69314718055994531f;
    lc = make_float2(0.5f * logf(ur * ur + ui * ui) + (float)e * kLn2, atan2f(ui, ur) + (float)(3.141592653589793 * h));
    const double den = sh.x * sh.x + sh.y * sh.y;
    th = make_float2((float)((ch.x * sh.x + ch.y * sh.y) / den), (float)((ch.y * sh.x - ch.x * sh.y) / den));
}

// log cosh z in double: the identities above next to a zero of cosh, elsewhere s z + log((1 + w)/2) with
// w = exp(-2 s z), s = sign Re z
__device__ __forceinline__ double2 log_cosh_double(double2 z) {
    double h;
    const double2 d = pole_offset(z, h);
    if (fabs(d.x) < 0.5 && fabs(d.y) < 0.5) {
        double2 sh, ch;
        sinh_cosh_small(d, sh, ch);
        return make_double2(0.5 * log(sh.x * sh.x + sh.y * sh.y), atan2(sh.y, sh.x) + 3.141592653589793 * h);
    }
    const double sg = z.x >= 0.0 ? 1.0 : -1.0;
    const double e = exp(-2.0 * fabs(z.x));
    double sn, cs;
    sincos(2.0 * sg * z.y, &sn, &cs);
    const double ur = 0.5 * (1.0 + e * cs), ui = -0.5 * e * sn;
    return make_double2(fabs(z.x) + 0.5 * log(ur * ur + ui * ui), sg * z.y + atan2(ui, ur));
}

// ---------------------------------------------------------------- log(2 cosh z), tanh z
// log(2 cosh z) = s z + log(1 + w), w = exp(-2 s z), s = sign(Re z), |w| <= 1.
__device__ __forceinline__ float2 log2cosh(float2 z) {
    const float s = z.x >= 0.f ? 1.f : -1.f;
    const float ax = fabsf(z.x), sy = s * z.y;
    const float e = expf(-2.f * ax);
    const float2 cs = cos_sin(2.f * sy);
    const float wr = e * cs.x, wi = -e * cs.y;
    return make_float2(ax + 0.5f * log1pf(2.f * wr + e * e), sy + atan2f(wi, 1.f + wr));
}
// Re log(2 cosh z) = |x| + log(q)/2, q = 1 + 2 e cos 2y + e^2 = |1 + e^{-2 s z}|^2 in [0, 4],
// e = exp(-2|x|), on the hardware transcendentals alone: v_exp_f32 (2^x), v_cos_f32 (cos 2 pi x,
// for |x| up to 256 revolutions, i.e. |y| < 804) and v_log_f32 (log2 x).
__device__ __forceinline__ float re_log2cosh_fast(float2 z) {
    constexpr float kM2Log2e = -2.8853900817779268f;  // exp(-2a) = 2^(-2a log2 e)
    constexpr float kInvPi = 0.31830988618379067f;    // cos 2y = cos(2 pi (y / pi))
    constexpr float kHalfLn2 = 0.34657359027997264f;  // log(q)/2 = (ln 2 / 2) log2 q
    const float ax = fabsf(z.x);
    const float e = __builtin_amdgcn_exp2f(ax * kM2Log2e);
    const float c = __builtin_amdgcn_cosf(z.y * kInvPi);
    const float q = fmaf(e, e, fmaf(2.f * e, c, 1.f));
    return fmaf(kHalfLn2, __builtin_amdgcn_logf(q), ax);
}
// tanh z = s (1 - w) / (1 + w), w = exp(-2 s z)
__device__ __forceinline__ float2 ctanhf(float2 z) {
    const float s = z.x >= 0.f ? 1.f : -1.f;
    const float e = expf(-2.f * fabsf(z.x));
    const float2 cs = cos_sin(2.f * s * z.y);
    const float wr = e * cs.x, wi = -e * cs.y;
    float2 q = cdiv(make_float2(1.f - wr, -wi), make_float2(1.f + wr, wi));
    return make_float2(s * q.x, s * q.y);
}

// ---------------------------------------------------------------- wave64 reductions
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}
__device__ __forceinline__ float2 wave_sum(float2 v) { return make_float2(wave_sum(v.x), wave_sum(v.y)); }
__device__ __forceinline__ double2 wave_sum(double2 v) { return make_double2(wave_sum(v.x), wave_sum(v.y)); }

// Sum over the wave, returned to every lane as a wave-uniform value.  DPP only (no
// LDS round trips): a butterfly over the 16 lanes of each row (quad swaps, then
// the half-row and row mirrors leave the row total in every lane of the row),
// then row broadcasts gather the four row totals into lane 63: (R3 + R2) +
// (R1 + R0).  The broadcasts write every row (rows 0 and 2 end with partial sums
// that lane 63 never reads), so each step is a single DPP add.  All 64 lanes
// must be active.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_move(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROW_MASK, 0xF, false));
}
__device__ __forceinline__ float wave_total(float v) {
    v += dpp_move<0xB1, 0xF>(v);   // quad_perm [1, 0, 3, 2]
    v += dpp_move<0x4E, 0xF>(v);   // quad_perm [2, 3, 0, 1]
    v += dpp_move<0x141, 0xF>(v);  // row_half_mirror
    v += dpp_move<0x140, 0xF>(v);  // row_mirror
    v += dpp_move<0x142, 0xF>(v);  // row_bcast:15: row 3 = R3 + R2, row 1 = R1 + R0
    v += dpp_move<0x143, 0xF>(v);  // row_bcast:31: row 3 += row 1
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ float uniform(float v) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

// Spin configuration spread over a wave: slot q of lane l holds site 64 q + l.
struct WaveSpins {
    int s[4];
    __device__ __forceinline__ void load(const int8_t* row, int N, int lane) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int site = q * kWave + lane;
            s[q] = site < N ? (int)row[site] : 0;
        }
    }
    __device__ __forceinline__ void store(int8_t* row, int N, int lane) const {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int site = q * kWave + lane;
            if (site < N) row[site] = (int8_t)s[q];
        }
    }
    // value of site i (i wave-uniform), broadcast to every lane; each slot is read with a constant
    // index and the choice is made among scalars, so s[] never needs an addressable copy
    __device__ __forceinline__ int get(int i) const {
        const int l = i & 63, q = i >> 6;
        const int v0 = __builtin_amdgcn_readlane(s[0], l), v1 = __builtin_amdgcn_readlane(s[1], l);
        const int v2 = __builtin_amdgcn_readlane(s[2], l), v3 = __builtin_amdgcn_readlane(s[3], l);
        return q == 0 ? v0 : q == 1 ? v1 : q == 2 ? v2 : v3;
    }
    __device__ __forceinline__ void set(int i, int value, int lane) {
        if ((i & 63) == lane) {
            const int q = i >> 6;
            s[0] = (q == 0) ? value : s[0];
            s[1] = (q == 1) ? value : s[1];
            s[2] = (q == 2) ? value : s[2];
            s[3] = (q == 3) ? value : s[3];
        }
    }
};

}  // namespace crbm
