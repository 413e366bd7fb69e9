// C-ABI layer of the chebrbm library: argument validation, plan and
// workspace management, and the launch sequence of every entry point.
// Nothing here synchronises the host; every launch goes to the caller's stream.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/chebrbm.h"
#include "internal.hpp"

namespace crbm {
hipError_t launch_local_core(const LocalArgs& A, const float2* th1, const float2* thn, const float2* thm,
                             hipStream_t stream);
hipError_t launch_lc_sums(const int8_t* sig, long n, int N, int M, const float2* a, const float2* b,
                          const float2* W, uint16_t* planes, float2* partial, const double2* Lg,
                          const double2* beta, double2* B, double2* Lg_out, hipStream_t stream);
hipError_t launch_fq_chunk(const Geometry& g, const int8_t* sig, long n_s, const double* q_host, int n_q,
                           double2* f, hipStream_t stream);
hipError_t launch_moment_accum(const double2* f, const double2* B, int b_is_f, const double* w, long n_s, int n_q,
                               int nn, int entry0, int total, double2* partial, int n_blocks, hipStream_t stream);
hipError_t launch_moment_final(const double2* partial, int n_blocks, int total, double2* mu, hipStream_t stream);
size_t sbuild_pack_bytes(int N, int M, long max_samples);
std::vector<int2> sbuild_order(int N, int M, int n_xcd, int g);
std::vector<int2> sbuild_order_ragged(int N, int M);
hipError_t launch_basis_pack(long n, const double2* B, const float2* loc, int mul, float2* Bcol, float2* HBcol,
                             hipStream_t stream);
long gram_partial_len(int K);
hipError_t launch_gram2(int K, long n, const float2* Bm, const float2* HBm, const double* w, double wdef,
                        double2* partial, double2* G, double2* H, int accumulate, hipStream_t stream);
hipError_t launch_sym_images(const int8_t* sig, long c, int N, int kind, int Lx, int Ly, int nrot, int8_t* img,
                             hipStream_t stream);
hipError_t launch_sym_combine(long rows, int ng, int N, const int8_t* img, int order0, const float2* lt,
                              const float2* el, const float2* lg, const double2* beta, float2* B, float2* HB,
                              hipStream_t stream);
hipError_t launch_sym_dft(long c, int K, int N, int kind, int Lx, int Ly, int nrot, const float2* B, const float2* HB,
                          float2* Bt, float2* HBt, hipStream_t stream);
hipError_t launch_correct(int K, const double2* G, const double2* H, double E_c, double W_scale, int n_out,
                          double2* work, double* mu, double* info, hipStream_t stream);
hipError_t launch_lanczos(int K, const double2* G, const double2* H, int n_steps, double2* work, double* a, double* b2,
                          double* info, hipStream_t stream);
hipError_t launch_spec_kpm(const double* mu, int n_mom, int jackson, double E0, double E_c, double W_scale,
                           const double* omega, int n_w, double* A, hipStream_t stream);
hipError_t launch_spec_cf(const double* a, const double* b2, int m, double E0, double eta, const double* omega,
                          int n_w, double* A, hipStream_t stream);
hipError_t launch_probe_mfma(int blocks, int iters, float* out, hipStream_t stream);
hipError_t launch_probe_copy(int blocks, const void* src, void* dst, long n16, hipStream_t stream);
hipError_t launch_probe_logcosh(int blocks, int iters, float* out, hipStream_t stream);
hipError_t launch_probe_gather(int blocks, const void* tab, int n_rows, int M, int iters, float* out,
                               hipStream_t stream);

}  // namespace crbm

using namespace crbm;

namespace {
constexpr int kMaxN = 256;
constexpr int kMaxM = 512;
constexpr int kQChunk = 8;
constexpr int kMomBlocks = 256;
constexpr int kMaxMomentEntries = 4096;   // n_q * (n_max + 1)
constexpr int kMaxBasis = 256;             // K = n_max + 1 of the moment-correction matrices
constexpr long kSplitBytes = 1L << 30;     // bound of the split-contraction buffer
constexpr long kMaxSplits = 12;
constexpr long kBorderSplitBytes = 256L << 20;   // bound of the border kernel's split slices
constexpr long kMaxBorderSplits = 16;
constexpr int kXcds = 8;                   // accelerator complex dies of the MI355X (round-robin dispatch)
#ifndef CRBM_SUPERTILE
#define CRBM_SUPERTILE 8
#endif
constexpr int kSuperTile = CRBM_SUPERTILE; // tile pairs per super-tile side in the S contraction order

thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}
int hip_fail(hipError_t e, const char* where) {
    return fail(CRBM_EHIP, "%s: %s", where, hipGetErrorString(e));
}
}  // namespace

struct crbm_plan_s {
    int device = 0;
    crbm_lattice lat{};
    int N = 0, M = 0;
    long P = 0;
    int n_bonds = 0;
    long max_samples = 0;
    int flags = 0;
    int2* bonds = nullptr;
    float4* bond_tab = nullptr;
    uint8_t* node_flag = nullptr;
    SrWork w{};
    float2* theta[3] = {nullptr, nullptr, nullptr};
    double2* momB = nullptr;
    double2* momF = nullptr;
    double2* mom_partial = nullptr;
    uint16_t* wplanes = nullptr;   // W split into 3 BF16 parts for the fused log-cosh sums
    double2* lcLg = nullptr;       // [max_samples] sum log cosh theta + a.sigma of psi_gs
    unsigned long long* bcounter = nullptr;
    unsigned long long* bclocks = nullptr;   // [CRBM_MAX_CLOCK_WAVES][2] per-wave clocks of the batched kernel
    double2* bpartial = nullptr;
    int n_cu = 256;
    int b_waves = 4, b_blocks = 1024, b_lanes = 64;
    Profiler prof;
    std::vector<void*> allocs;
    // workspace of the moment-correction path, reserved at creation (CRBM_PLAN_BASIS / CRBM_PLAN_SYM_BASIS;
    // the small dense buffer of the corrected moments and Lanczos in every plan); the calls check its size
    enum { GB_BASIS = 0, GB_HBASIS, GB_ELOC, GB_GRAM, GB_SMALL, GB_SYMIMG, GB_SYMLT, GB_SYMLG, GB_SYMBT, GB_SYMHBT,
           GB_COUNT };
    void* grow_ptr[GB_COUNT] = {};
    size_t grow_cap[GB_COUNT] = {};
    int basis_k_max = 0;

    Geometry geometry() const {
        Geometry g;
        g.N = N; g.M = M; g.P = (int)P; g.n_bonds = n_bonds; g.bonds = bonds;
        g.kind = lat.kind; g.Lx = lat.Lx; g.J = lat.J;
        g.bond_tab = bond_tab;
        g.node_flag = node_flag;
        return g;
    }
    template <class T>
    int alloc(T** p, size_t count) {
        void* q = nullptr;
        if (count == 0) count = 1;
        hipError_t e = hipMalloc(&q, count * sizeof(T));
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(CRBM_ENOMEM, "hipMalloc of %zu bytes failed: %s", count * sizeof(T), hipGetErrorString(e));
        }
        allocs.push_back(q);
        *p = static_cast<T*>(q);
        return CRBM_OK;
    }
    // reserve grow_ptr[id] with `bytes` (at plan creation only)
    int reserve(int id, size_t bytes) {
        if (grow_cap[id] >= bytes) return CRBM_OK;
        if (grow_ptr[id]) { (void)hipFree(grow_ptr[id]); grow_ptr[id] = nullptr; grow_cap[id] = 0; }
        void* q = nullptr;
        hipError_t e = hipMalloc(&q, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(CRBM_ENOMEM, "hipMalloc of %zu bytes failed: %s", bytes, hipGetErrorString(e));
        }
        grow_ptr[id] = q;
        grow_cap[id] = bytes;
        return CRBM_OK;
    }
    // the calls: the reserved buffer must hold `bytes`
    int need(int id, size_t bytes, const char* flag) const {
        if (grow_cap[id] >= bytes) return CRBM_OK;
        return fail(CRBM_ENOMEM, "the plan's basis workspace holds %zu bytes where %zu are needed: create the plan with "
                    "crbm_plan_create_ex, %s and basis_k_max >= K", grow_cap[id], bytes, flag);
    }
    ~crbm_plan_s() {
        for (void* p : allocs) (void)hipFree(p);
        for (void* p : grow_ptr)
            if (p) (void)hipFree(p);
    }
};

namespace {
// Upper bound on the sample chunks of the O^H c contraction for any n <= max_samples:
// chunks of at least 256 samples and at least n/256 samples, so at most min(ceil(n/256), 257).
long ot_chunks_bound(long max_samples) {
    const long c = (max_samples + 255) / 256;
    return c < 257 ? c : 257;
}

int check_rbm(const crbm_plan_s* p, const crbm_rbm* r, const char* name) {
    if (!r) return fail(CRBM_EINVAL, "%s is NULL", name);
    if (!r->a || !r->b || !r->W) return fail(CRBM_EINVAL, "%s has a NULL parameter array", name);
    if (r->n_visible != p->N || r->n_hidden != p->M)
        return fail(CRBM_EINVAL, "%s has shape (N=%d, M=%d) but the plan has (N=%d, M=%d)", name, r->n_visible,
                    r->n_hidden, p->N, p->M);
    return CRBM_OK;
}

// principal complex logarithm of a complex double, rounded to binary32 (log 0 = -inf)
float2 log_of(double2 z) {
    return make_float2((float)std::log(std::hypot(z.x, z.y)), (float)std::atan2(z.y, z.x));
}

RbmView view(const crbm_rbm* r) {
    RbmView v;
    v.a = static_cast<const float2*>(r->a);
    v.b = static_cast<const float2*>(r->b);
    v.W = static_cast<const float2*>(r->W);
    return v;
}

int check_plan(crbm_plan p) {
    if (!p) return fail(CRBM_EINVAL, "plan is NULL");
    return CRBM_OK;
}

int set_device(crbm_plan p) {
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (cur != p->device) return fail(CRBM_EINVAL, "plan was created on device %d but device %d is current",
                                      p->device, cur);
    return CRBM_OK;
}
}  // namespace

namespace {
// milliseconds of one launch sequence timed with events on `stream` (synchronises), or < 0 on error
template <class F>
double timed_ms(hipStream_t stream, F&& launch) {
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return -1.0;
    if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return -1.0; }
    float ms = -1.f;
    hipError_t r = hipEventRecord(e0, stream);
    if (r == hipSuccess) r = launch();
    if (r == hipSuccess) r = hipEventRecord(e1, stream);
    if (r == hipSuccess) r = hipEventSynchronize(e1);
    if (r == hipSuccess) r = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return r == hipSuccess ? (double)ms : -1.0;
}
int current_cus() {
    int dev = 0, n_cu = 256;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n_cu < 1) n_cu = 256;
    return n_cu;
}
}  // namespace

extern "C" {

const char* crbm_last_error(void) { return g_err; }

int crbm_plan_create(crbm_plan* out, const crbm_lattice* lat, int n_hidden, long max_samples, int flags) {
    return crbm_plan_create_ex(out, lat, n_hidden, max_samples, flags, 0);
}

int crbm_plan_create_ex(crbm_plan* out, const crbm_lattice* lat, int n_hidden, long max_samples, int flags,
                        int basis_k_max) {
    if (!out) return fail(CRBM_EINVAL, "plan output pointer is NULL");
    *out = nullptr;
    if (!lat) return fail(CRBM_EINVAL, "lattice is NULL");
    if (lat->kind != CRBM_LATTICE_CHAIN && lat->kind != CRBM_LATTICE_SQUARE)
        return fail(CRBM_EINVAL, "unknown lattice kind %d", lat->kind);
    const int Ly = lat->kind == CRBM_LATTICE_CHAIN ? 1 : lat->Ly;
    if (lat->Lx < 2 || Ly < 1 || (lat->kind == CRBM_LATTICE_SQUARE && Ly < 2))
        return fail(CRBM_EINVAL, "lattice sides must be >= 2 (got Lx=%d, Ly=%d)", lat->Lx, Ly);
    const long N = (long)lat->Lx * Ly;
    if (N > kMaxN) return fail(CRBM_EUNSUPPORTED, "N = %ld sites exceeds the limit of %d", N, kMaxN);
    if (n_hidden < 1) return fail(CRBM_EINVAL, "n_hidden must be >= 1 (got %d)", n_hidden);
    if (n_hidden > kMaxM) return fail(CRBM_EUNSUPPORTED, "M = %d hidden units exceeds the limit of %d", n_hidden, kMaxM);
    if (max_samples < 1) return fail(CRBM_EINVAL, "max_samples must be >= 1 (got %ld)", max_samples);
    if (flags & ~(CRBM_PLAN_DENSE_S | CRBM_PLAN_CHOLESKY | CRBM_PLAN_BASIS | CRBM_PLAN_SYM_BASIS))
        return fail(CRBM_EINVAL, "unknown plan flags 0x%x", flags);
    const bool basis = (flags & (CRBM_PLAN_BASIS | CRBM_PLAN_SYM_BASIS)) != 0;
    if (basis && (basis_k_max < 1 || basis_k_max > kMaxBasis))
        return fail(CRBM_EINVAL, "basis_k_max must be in [1, %d] with CRBM_PLAN_BASIS (got %d)", kMaxBasis, basis_k_max);

    crbm_plan_s* p = new (std::nothrow) crbm_plan_s();
    if (!p) return fail(CRBM_ENOMEM, "host allocation of the plan failed");
    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) { delete p; return hip_fail(e, "hipGetDevice"); }
    p->lat = *lat;
    p->lat.Ly = Ly;
    p->N = (int)N;
    p->M = n_hidden;
    p->P = N + n_hidden + N * n_hidden;
    p->max_samples = max_samples;
    p->flags = flags;
    if ((flags & CRBM_PLAN_CHOLESKY) && p->P > kCholMaxP) {
        delete p;
        return fail(CRBM_EUNSUPPORTED, "CRBM_PLAN_CHOLESKY needs P <= %ld (P = %ld)", kCholMaxP, N + n_hidden + N * n_hidden);
    }

    // bonds of the periodic lattice (Sec. VI)
    std::vector<int2> bonds;
    if (lat->kind == CRBM_LATTICE_CHAIN) {
        for (int i = 0; i < lat->Lx; ++i) bonds.push_back(make_int2(i, (i + 1) % lat->Lx));
    } else {
        for (int y = 0; y < Ly; ++y)
            for (int x = 0; x < lat->Lx; ++x) {
                const int r = x + lat->Lx * y;
                bonds.push_back(make_int2(r, (x + 1) % lat->Lx + lat->Lx * y));
                bonds.push_back(make_int2(r, x + lat->Lx * ((y + 1) % Ly)));
            }
    }
    p->n_bonds = (int)bonds.size();
    if (p->n_bonds > kMaxBonds) {
        delete p;
        return fail(CRBM_EUNSUPPORTED, "%d bonds exceed the limit of %d", (int)bonds.size(), kMaxBonds);
    }

    const long P = p->P, M = n_hidden, S = max_samples;
    const long plane = (N + 1) * (M + 1);
    const long red_len = ot_chunks_bound(S) * 2 * plane + 2048;
    int rc = CRBM_OK;
    rc = rc ? rc : p->alloc(&p->bonds, bonds.size());
    rc = rc ? rc : p->alloc(&p->bond_tab, bonds.size() * (size_t)n_hidden);
    rc = rc ? rc : p->alloc(&p->node_flag, S);
    rc = rc ? rc : p->alloc(&p->w.scal, 32);
    rc = rc ? rc : p->alloc(&p->w.Om, P);
    rc = rc ? rc : p->alloc(&p->w.Om16, P);
    rc = rc ? rc : p->alloc(&p->w.ORm, P);
    rc = rc ? rc : p->alloc(&p->w.F, P);
    rc = rc ? rc : p->alloc(&p->w.x, P);
    rc = rc ? rc : p->alloc(&p->w.r, P);
    rc = rc ? rc : p->alloc(&p->w.p, P);
    rc = rc ? rc : p->alloc(&p->w.Ap, P);
    rc = rc ? rc : p->alloc(&p->w.vstage, P);
    rc = rc ? rc : p->alloc(&p->w.u, S);
    rc = rc ? rc : p->alloc(&p->w.red, red_len);
    // G: the matrix-free product's O v partials, ceil(M / 64) double2 (2 ceil(M / 64) float2) per sample
    rc = rc ? rc : p->alloc(&p->w.G, S * 2 * ((M + 63) / 64));
    rc = rc ? rc : p->alloc(&p->w.sig16, S * (long)sig16_row(N));
    for (int k = 0; k < 3 && !rc; ++k) rc = p->alloc(&p->theta[k], S * M);
    rc = rc ? rc : p->alloc(&p->momB, S);
    rc = rc ? rc : p->alloc(&p->momF, (long)kQChunk * S);
    rc = rc ? rc : p->alloc(&p->mom_partial, (long)kMomBlocks * kMaxMomentEntries);
    rc = rc ? rc : p->alloc(&p->wplanes, lc_plane_elems(N, M));
    p->w.wplanes = p->wplanes;
    rc = rc ? rc : p->alloc(&p->lcLg, S);
    rc = rc ? rc : p->alloc(&p->bcounter, 1);
    rc = rc ? rc : p->alloc(&p->bclocks, (size_t)2 * CRBM_MAX_CLOCK_WAVES);
    rc = rc ? rc : p->alloc(&p->bpartial, 2 * S);
    if (!rc && (flags & (CRBM_PLAN_DENSE_S | CRBM_PLAN_CHOLESKY))) {
        rc = p->alloc(&p->w.S, P * P);
        const long nT = hemv_tiles(P);
        rc = rc ? rc : p->alloc(&p->w.hv_part, nT * nT * kHemvTile);
    }
    if (!rc && (flags & CRBM_PLAN_CHOLESKY)) rc = p->alloc(&p->w.S64, P * P);
    std::vector<int2> order;
    if (!rc && (flags & (CRBM_PLAN_DENSE_S | CRBM_PLAN_CHOLESKY))) {
        p->w.pack_bytes = sbuild_pack_bytes((int)N, (int)M, S);
        rc = p->alloc(reinterpret_cast<unsigned char**>(&p->w.pack), p->w.pack_bytes);
        // the pairs of full tiles, then the ragged pairs of the last site block (one launch takes both)
        order = sbuild_order((int)N, (int)M, kXcds, kSuperTile);
        const std::vector<int2> rag = sbuild_order_ragged((int)N, (int)M);
        order.insert(order.end(), rag.begin(), rag.end());
        int2* d_order = nullptr;
        rc = rc ? rc : p->alloc(&d_order, order.size());
        p->w.sb_order = d_order;
        p->w.sb_order_len = (long)order.size();
        // buffer of a contraction split over samples when the tile pairs alone cannot fill the device
        const long slice = P * P * (long)sizeof(float2);
        const long nsm = std::min<long>(kMaxSplits, kSplitBytes / slice);
        if (!rc && nsm >= 2) {
            rc = p->alloc(&p->w.spart, (size_t)(nsm * P * P));
            p->w.nsplit_max = (int)nsm;
        }
        // slices of the border kernel split over samples (at least as many as the tile pairs use)
        const long nsb = std::min<long>(kMaxBorderSplits, kBorderSplitBytes / (N * P * (long)sizeof(float2)));
        p->w.nsb_max = 1;
        if (!rc && nsb >= 2) {
            rc = p->alloc(&p->w.bx_part, (size_t)(nsb * N * P));
            p->w.nsb_max = (int)nsb;
        }
        rc = rc ? rc : p->alloc(&p->w.bx, (size_t)(N * P));
    }
    // small dense buffer of the corrected moments and Lanczos (K <= 256), in every plan
    rc = rc ? rc : p->reserve(crbm_plan_s::GB_SMALL, (size_t)(4L * kMaxBasis * kMaxBasis + kMaxBasis) * sizeof(double2));
    if (!rc && basis) {
        const size_t col = (size_t)basis_k_max * (size_t)S * sizeof(float2);
        p->basis_k_max = basis_k_max;
        rc = p->reserve(crbm_plan_s::GB_BASIS, col);
        rc = rc ? rc : p->reserve(crbm_plan_s::GB_HBASIS, col);
        rc = rc ? rc : p->reserve(crbm_plan_s::GB_ELOC, (size_t)S * sizeof(float2));
        long gl = 0;   // the Gram partials' length is not monotone in K: the largest up to K_max
        for (int k = 1; k <= basis_k_max; ++k) gl = std::max(gl, gram_partial_len(k));
        rc = rc ? rc : p->reserve(crbm_plan_s::GB_GRAM, (size_t)gl * sizeof(double2));
        if (!rc && (flags & CRBM_PLAN_SYM_BASIS)) {
            rc = p->reserve(crbm_plan_s::GB_SYMBT, col);
            rc = rc ? rc : p->reserve(crbm_plan_s::GB_SYMHBT, col);
            rc = rc ? rc : p->reserve(crbm_plan_s::GB_SYMIMG, (size_t)S * (size_t)N);
            rc = rc ? rc : p->reserve(crbm_plan_s::GB_SYMLT, (size_t)S * sizeof(float2));
            rc = rc ? rc : p->reserve(crbm_plan_s::GB_SYMLG, (size_t)S * sizeof(float2));
        }
    }
    p->w.prof = &p->prof;
    if (rc) { delete p; return rc; }
    p->w.red_len = red_len;
    if (hipDeviceGetAttribute(&p->n_cu, hipDeviceAttributeMultiprocessorCount, p->device) != hipSuccess || p->n_cu < 1)
        p->n_cu = 256;
    p->b_waves = 4;
    p->b_blocks = 4 * p->n_cu;
    p->w.n_cu = p->n_cu;
    p->w.sb_kt = 128;
    e = hipMemcpy(p->bonds, bonds.data(), bonds.size() * sizeof(int2), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(p->w.scal, 0, 32 * sizeof(double));
    if (e == hipSuccess && !order.empty())
        e = hipMemcpy(const_cast<int2*>(p->w.sb_order), order.data(), order.size() * sizeof(int2),
                      hipMemcpyHostToDevice);
    if (e != hipSuccess) { delete p; return hip_fail(e, "plan initialisation"); }
    *out = p;
    return CRBM_OK;
}

int crbm_plan_destroy(crbm_plan plan) {
    if (!plan) return fail(CRBM_EINVAL, "plan is NULL");
    delete plan;
    return CRBM_OK;
}

int crbm_plan_buffer(crbm_plan p, int which, void** ptr, size_t* bytes) {
    if (check_plan(p)) return CRBM_EINVAL;
    if (!ptr) return fail(CRBM_EINVAL, "dev_ptr is NULL");
    size_t b = 0;
    switch (which) {
        case CRBM_BUF_F: *ptr = p->w.F; b = p->P * sizeof(double2); break;
        case CRBM_BUF_DALPHA: *ptr = p->w.x; b = p->P * sizeof(double2); break;
        case CRBM_BUF_OMEAN: *ptr = p->w.Om; b = p->P * sizeof(double2); break;
        case CRBM_BUF_S:
            if (!p->w.S) return fail(CRBM_EINVAL, "the plan holds no dense S (create it with CRBM_PLAN_DENSE_S)");
            *ptr = p->w.S; b = p->P * p->P * sizeof(float2); break;
        case CRBM_BUF_WAVE_CLOCKS:
            *ptr = p->bclocks; b = (size_t)CRBM_MAX_CLOCK_WAVES * 2 * sizeof(unsigned long long); break;
        default: return fail(CRBM_EINVAL, "unknown buffer id %d", which);
    }
    if (bytes) *bytes = b;
    return CRBM_OK;
}

int crbm_plan_profile(crbm_plan p, int enable) {
    if (check_plan(p)) return CRBM_EINVAL;
    if (enable != 0 && enable != 1) return fail(CRBM_EINVAL, "enable must be 0 or 1");
    p->prof.reset();
    p->prof.on = enable != 0;
    return CRBM_OK;
}

int crbm_plan_profile_read(crbm_plan p, int group, int* count, double* total_ms) {
    if (check_plan(p)) return CRBM_EINVAL;
    if (group < 0 || group >= PROF_COUNT) return fail(CRBM_EINVAL, "unknown profile group %d", group);
    int c = 0;
    double t = 0.0;
    for (const auto& r : p->prof.recs) {
        if (r.id != group) continue;
        hipError_t e = hipEventSynchronize(r.b);
        if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, r.a, r.b);
        if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
        ++c;
        t += ms;
    }
    if (count) *count = c;
    if (total_ms) *total_ms = t;
    return CRBM_OK;
}

int crbm_init_rbm(const crbm_rbm* r, uint64_t seed, float stddev, hipStream_t stream) {
    if (!r || !r->a || !r->b || !r->W) return fail(CRBM_EINVAL, "rbm or one of its arrays is NULL");
    if (r->n_visible < 1 || r->n_hidden < 1) return fail(CRBM_EINVAL, "rbm sizes must be >= 1");
    if (!(stddev >= 0.f)) return fail(CRBM_EINVAL, "stddev must be >= 0");
    hipError_t e = launch_init_rbm((float2*)r->a, (float2*)r->b, (float2*)r->W, r->n_visible, r->n_hidden, seed,
                                   stddev, stream);
    return e == hipSuccess ? CRBM_OK : hip_fail(e, "init_rbm launch");
}

int crbm_init_chains(crbm_plan p, int8_t* spins, int n_chains, uint64_t seed, int zero_mag, hipStream_t stream) {
    if (check_plan(p)) return CRBM_EINVAL;
    if (!spins) return fail(CRBM_EINVAL, "spins is NULL");
    if (n_chains < 1) return fail(CRBM_EINVAL, "n_chains must be >= 1");
    if (zero_mag != 0 && zero_mag != 1) return fail(CRBM_EINVAL, "zero_magnetisation must be 0 or 1");
    if (zero_mag && (p->N % 2)) return fail(CRBM_EINVAL, "zero magnetisation needs an even number of sites");
    if (int rc = set_device(p)) return rc;
    hipError_t e = launch_init_chains(spins, p->N, n_chains, seed, zero_mag, stream);
    return e == hipSuccess ? CRBM_OK : hip_fail(e, "init_chains launch");
}

int crbm_sample(crbm_plan p, const crbm_rbm* psi, int8_t* spins, void* theta_out, void* logpsi_out, int n_chains,
                int n_sweeps, int proposal, uint64_t seed, uint64_t step_offset, int8_t* samples_out,
                uint32_t* n_accept, uint32_t* accept_trace, hipStream_t stream) {
    if (check_plan(p)) return CRBM_EINVAL;
    if (int rc = check_rbm(p, psi, "psi")) return rc;
    if (!spins) return fail(CRBM_EINVAL, "spins is NULL");
    if (n_chains < 1) return fail(CRBM_EINVAL, "n_chains must be >= 1");
    if (n_sweeps < 0) return fail(CRBM_EINVAL, "n_sweeps must be >= 0");
    if (proposal != CRBM_PROPOSAL_FLIP && proposal != CRBM_PROPOSAL_EXCHANGE)
        return fail(CRBM_EINVAL, "unknown proposal %d", proposal);
    if (int rc = set_device(p)) return rc;
    SampleArgs A;
    A.psi = view(psi);
    A.N = p->N;
    A.M = p->M;
    A.spins = spins;
    A.theta_out = static_cast<float2*>(theta_out);
    A.logpsi_out = static_cast<float2*>(logpsi_out);
    A.n_chains = n_chains;
    A.n_sweeps = n_sweeps;
    A.proposal = proposal;
    A.seed = seed;
    A.step_offset = step_offset;
    A.samples_out = samples_out;
    A.n_accept = n_accept;
    A.trace = accept_trace;
    A.trace_words = (int)(((long)n_sweeps * p->N + 31) / 32);
    p->prof.begin(PROF_SAMPLE, stream);
    hipError_t e = launch_sample(A, stream);
    p->prof.end(stream);
    return e == hipSuccess ? CRBM_OK : hip_fail(e, "sample launch");
}

int crbm_local_estimators(crbm_plan p, const crbm_rbm* fit, const crbm_rbm* psi_n, const crbm_rbm* psi_nm1,
                          const crbm_cheb* cheb, const int8_t* samples, long n, void* logpsi_out, void* eloc_out,
                          void* R_out, void* tanh_out, void* O_out, hipStream_t stream) {
    if (check_plan(p)) return CRBM_EINVAL;
    if (int rc = check_rbm(p, fit, "fit")) return rc;
    if (n < 0) return fail(CRBM_EINVAL, "n_samples must be >= 0");
    if (n > 0 && !samples) return fail(CRBM_EINVAL, "samples is NULL");
    if (n > p->max_samples) return fail(CRBM_ENOMEM, "n_samples = %ld exceeds the plan's max_samples = %ld", n,
                                        p->max_samples);
    const bool cheb_mode = psi_n != nullptr;
    if (cheb_mode) {
        if (!cheb) return fail(CRBM_EINVAL, "cheb is NULL in Chebyshev mode");
        if (int rc = check_rbm(p, psi_n, "psi_n")) return rc;
        if (cheb->order < 0) return fail(CRBM_EINVAL, "order must be >= 0");
        if (cheb->order >= 1)
            if (int rc = check_rbm(p, psi_nm1, "psi_nm1")) return rc;
        if (!(cheb->W_scale != 0.0)) return fail(CRBM_EINVAL, "W_scale must be non-zero");
    } else if (R_out) {
        return fail(CRBM_EINVAL, "R_out needs Chebyshev mode (psi_n != NULL)");
    }
    if (int rc = set_device(p)) return rc;
    if (n == 0) return CRBM_OK;

    LocalArgs A{};
    A.g = p->geometry();
    A.fit = view(fit);
    A.cheb_mode = cheb_mode;
    if (cheb_mode) {
        A.psn = view(psi_n);
        if (cheb->order >= 1) A.psm = view(psi_nm1);
        A.order = cheb->order;
        A.E_c = cheb->E_c;
        A.W_scale = cheb->W_scale;
        A.beta_n = make_double2(cheb->beta_n[0], cheb->beta_n[1]);
        A.beta_nm1 = make_double2(cheb->beta_nm1[0], cheb->beta_nm1[1]);
        A.lbeta_n = log_of(A.beta_n);
        A.lbeta_nm1 = log_of(A.beta_nm1);
        A.q0 = cheb->q[0];
        A.q1 = p->lat.kind == CRBM_LATTICE_CHAIN ? 0.0 : cheb->q[1];
    }
    A.samples = samples;
    A.n_samples = n;
    A.logpsi_out = static_cast<float2*>(logpsi_out);
    A.eloc_out = static_cast<float2*>(eloc_out);
    A.R_out = static_cast<float2*>(R_out);
    A.tanh_out = static_cast<float2*>(tanh_out);
    A.O_out = static_cast<float2*>(O_out);
    auto theta = [&](const RbmView& v, float2* out) {
        p->prof.begin(PROF_THETA, stream);
        hipError_t r = launch_theta(samples, n, p->N, p->M, v.b, v.W, out, p->wplanes, stream);
        p->prof.end(stream);
        return r;
    };
    hipError_t e = theta(A.fit, p->theta[0]);
    if (e == hipSuccess && cheb_mode) e = theta(A.psn, p->theta[1]);
    if (e == hipSuccess && cheb_mode && cheb->order >= 1) e = theta(A.psm, p->theta[2]);
    if (e == hipSuccess) {
        p->prof.begin(PROF_LOCAL, stream);
        e = launch_local_core(A, p->theta[0], p->theta[1], p->theta[2], stream);
        p->prof.end(stream);
    }
    return e == hipSuccess ? CRBM_OK : hip_fail(e, "local_estimators launch");
}

static int sr_step_common(crbm_plan p, const crbm_rbm* fit, const int8_t* samples, const double* weights,
                          const void* T, const void* R, long n, double dgamma, double eps, int solver, int prec,
                          double cg_tol, int cg_maxit, double* stats_out, int mode, hipStream_t stream) {
    if (check_plan(p)) return CRBM_EINVAL;
    if (int rc = check_rbm(p, fit, "fit")) return rc;
    if (!samples || !T || !R)
        return fail(CRBM_EINVAL, mode == 1 ? "samples, tanh_theta and eloc must be non-NULL"
                                           : "samples, tanh_theta and R must be non-NULL");
    if (mode == 1 && !(dgamma - dgamma == 0.0)) return fail(CRBM_EINVAL, "lr must be finite");
    if (n < 1) return fail(CRBM_EINVAL, "n_samples must be >= 1");
    if (n > p->max_samples) return fail(CRBM_ENOMEM, "n_samples = %ld exceeds the plan's max_samples = %ld", n,
                                        p->max_samples);
    if (solver != CRBM_SOLVER_CG_DENSE && solver != CRBM_SOLVER_CG_MATFREE && solver != CRBM_SOLVER_CHOLESKY)
        return fail(CRBM_EINVAL, "unknown solver %d", solver);
    if (prec != CRBM_PREC_FP32 && prec != CRBM_PREC_BF16) return fail(CRBM_EINVAL, "unknown precision %d", prec);
    if (prec == CRBM_PREC_BF16 && weights && solver != CRBM_SOLVER_CG_MATFREE)
        return fail(CRBM_EUNSUPPORTED, "the BF16 S contraction needs uniform weights (weights == NULL)");
    if (!(eps >= 0.0)) return fail(CRBM_EINVAL, "diag_shift must be >= 0");
    if (solver != CRBM_SOLVER_CHOLESKY && (cg_maxit < 1 || !(cg_tol > 0.0)))
        return fail(CRBM_EINVAL, "cg_maxit must be >= 1 and cg_tol > 0");
    if (solver == CRBM_SOLVER_CG_DENSE && !p->w.S)
        return fail(CRBM_EINVAL, "CG_DENSE needs a plan created with CRBM_PLAN_DENSE_S");
    if (solver == CRBM_SOLVER_CHOLESKY && !p->w.S64)
        return fail(CRBM_EINVAL, "CHOLESKY needs a plan created with CRBM_PLAN_CHOLESKY");
    if (int rc = set_device(p)) return rc;
    SrArgs A{};
    A.N = p->N; A.M = p->M; A.P = (int)p->P;
    A.a = (float2*)fit->a; A.b = (float2*)fit->b; A.W = (float2*)fit->W;
    A.samples = samples;
    A.weights = weights;
    A.T = static_cast<const float2*>(T);
    A.R = static_cast<const float2*>(R);
    A.n = n;
    A.dgamma = dgamma;
    A.eps = eps;
    A.solver = solver;
    A.prec = prec;
    A.cg_tol = cg_tol;
    A.cg_maxit = solver == CRBM_SOLVER_CHOLESKY ? 0 : cg_maxit;
    A.stats = stats_out;
    A.mode = mode;
    hipError_t e = launch_sr_step(A, p->w, stream);
    return e == hipSuccess ? CRBM_OK : hip_fail(e, "sr_step launch");
}

int crbm_sr_step(crbm_plan p, const crbm_rbm* fit, const int8_t* samples, const double* weights, const void* T,
                 const void* R, long n, double dgamma, double eps, int solver, int prec, double cg_tol, int cg_maxit,
                 double* stats_out, hipStream_t stream) {
    return sr_step_common(p, fit, samples, weights, T, R, n, dgamma, eps, solver, prec, cg_tol, cg_maxit, stats_out,
                          0, stream);
}

int crbm_sr_energy_step(crbm_plan p, const crbm_rbm* psi, const int8_t* samples, const double* weights, const void* T,
                        const void* eloc, long n, double lr, double eps, int solver, int prec, double cg_tol,
                        int cg_maxit, double* stats_out, hipStream_t stream) {
    return sr_step_common(p, psi, samples, weights, T, eloc, n, -lr, eps, solver, prec, cg_tol, cg_maxit, stats_out,
                          1, stream);
}

int crbm_fit_stats(crbm_plan p, const void* R, const double* weights, long n, double* stats_out, hipStream_t stream) {
    if (check_plan(p)) return CRBM_EINVAL;
    if (!R || !stats_out) return fail(CRBM_EINVAL, "R and stats_out must be non-NULL");
    if (n < 1) return fail(CRBM_EINVAL, "n_samples must be >= 1");
    if (int rc = set_device(p)) return rc;
    hipError_t e = launch_fit_stats(static_cast<const float2*>(R), weights, n, p->w.red, stats_out, stream);
    return e == hipSuccess ? CRBM_OK : hip_fail(e, "fit_stats launch");
}

int crbm_enum_weights(crbm_plan p, const void* logpsi, long n, double* weights_out, hipStream_t stream) {
    if (check_plan(p)) return CRBM_EINVAL;
    if (!logpsi || !weights_out) return fail(CRBM_EINVAL, "logpsi and weights_out must be non-NULL");
    if (n < 1) return fail(CRBM_EINVAL, "n must be >= 1");
    if (int rc = set_device(p)) return rc;
    hipError_t e = launch_enum_weights(static_cast<const float2*>(logpsi), n, p->w.red, weights_out, stream);
    return e == hipSuccess ? CRBM_OK : hip_fail(e, "enum_weights launch");
}

int crbm_chebyshev_moment(crbm_plan p, const crbm_rbm* gs, const void* t_params, const double* betas, int n_max,
                          const double* q, int n_q, const int8_t* samples, const double* weights, long n,
                          void* mu_out, hipStream_t stream) {
    if (check_plan(p)) return CRBM_EINVAL;
    if (int rc = check_rbm(p, gs, "psi_gs")) return rc;
    if (n_max < 0) return fail(CRBM_EINVAL, "n_max must be >= 0");
    if (n_max > 0 && (!t_params || !betas)) return fail(CRBM_EINVAL, "t_params and betas must be non-NULL");
    if (n_q < 1 || !q) return fail(CRBM_EINVAL, "need n_q >= 1 momenta");
    if ((long)n_q * (n_max + 1) > kMaxMomentEntries)
        return fail(CRBM_EUNSUPPORTED, "n_q * (n_max + 1) = %ld exceeds %d", (long)n_q * (n_max + 1),
                    kMaxMomentEntries);
    if (!samples || !mu_out) return fail(CRBM_EINVAL, "samples and mu_out must be non-NULL");
    if (n < 1) return fail(CRBM_EINVAL, "n_samples must be >= 1");
    if (n > p->max_samples) return fail(CRBM_ENOMEM, "n_samples = %ld exceeds the plan's max_samples = %ld", n,
                                        p->max_samples);
    if (int rc = set_device(p)) return rc;
    const Geometry g = p->geometry();
    const RbmView vg = view(gs);
    const int nn = n_max + 1;
    const long P = p->P;
    const float2* tp = static_cast<const float2*>(t_params);
    // per-sample sum log cosh theta + a.sigma of psi_gs, once; the tile partials go to theta[2]
    p->prof.begin(PROF_MOMENT, stream);
    hipError_t e = launch_lc_sums(samples, n, p->N, p->M, vg.a, vg.b, vg.W, p->wplanes, p->theta[2], nullptr,
                                  nullptr, nullptr, p->lcLg, stream);
    p->prof.end(stream);
    for (int q0 = 0; q0 < n_q && e == hipSuccess; q0 += kQChunk) {
        const int nq = (n_q - q0) < kQChunk ? (n_q - q0) : kQChunk;
        e = launch_fq_chunk(g, samples, n, q + 2 * q0, nq, p->momF, stream);
        if (e == hipSuccess)
            e = launch_moment_accum(p->momF, nullptr, 1, weights, n, nq, nn, q0 * nn, nn * n_q, p->mom_partial,
                                    kMomBlocks, stream);
        for (int t = 1; t <= n_max && e == hipSuccess; ++t) {
            const float2* at = tp + (long)(t - 1) * P;
            // B_t = beta_t t~_t / psi_gs from the fused product and log-cosh sums
            p->prof.begin(PROF_MOMENT, stream);
            e = launch_lc_sums(samples, n, p->N, p->M, at, at + p->N, at + p->N + p->M, p->wplanes, p->theta[2],
                               p->lcLg, reinterpret_cast<const double2*>(betas) + (t - 1), p->momB, nullptr, stream);
            p->prof.end(stream);
            if (e == hipSuccess)
                e = launch_moment_accum(p->momF, p->momB, 0, weights, n, nq, nn, q0 * nn + t, nn * n_q,
                                        p->mom_partial, kMomBlocks, stream);
        }
    }
    if (e == hipSuccess)
        e = launch_moment_final(p->mom_partial, kMomBlocks, nn * n_q, static_cast<double2*>(mu_out), stream);
    return e == hipSuccess ? CRBM_OK : hip_fail(e, "chebyshev_moment launch");
}

int crbm_fidelity_grad(crbm_plan p, const crbm_rbm* fit, const int8_t* samples, const void* T, const void* R, long n,
                       void* grad_out, double* loss_out, hipStream_t stream) {
    if (check_plan(p)) return CRBM_EINVAL;
    if (int rc = check_rbm(p, fit, "fit")) return rc;
    if (!samples || !T || !R) return fail(CRBM_EINVAL, "samples, tanh_theta and R must be non-NULL");
    if (!grad_out && !loss_out) return fail(CRBM_EINVAL, "at least one of grad_out and loss_out must be non-NULL");
    if (n < 1) return fail(CRBM_EINVAL, "n_samples must be >= 1");
    if (n > p->max_samples) return fail(CRBM_ENOMEM, "n_samples = %ld exceeds the plan's max_samples = %ld", n,
                                        p->max_samples);
    if (int rc = set_device(p)) return rc;
    GradArgs A{};
    A.N = p->N; A.M = p->M; A.P = (int)p->P;
    A.samples = samples;
    A.T = static_cast<const float2*>(T);
    A.R = static_cast<const float2*>(R);
    A.n = n;
    A.grad = static_cast<double2*>(grad_out);
    A.loss = loss_out;
    hipError_t e = launch_fidelity_grad(A, p->w, stream);
    return e == hipSuccess ? CRBM_OK : hip_fail(e, "fidelity_grad launch");
}

}  // extern "C"

// ------------------------------------------------------------------ allocation-free fidelity gradient
// The scratch of crbm_fidelity_grad_noalloc: one file-scope device array, which every GPU the library runs on
// holds until the process ends.  Host code never passes the array's name (a host-side stand-in) to a kernel:
// its device address is taken once per device with hipGetSymbolAddress and kept in g_scratch_ptr.
namespace {
constexpr size_t kNoallocScratchBytes = size_t(48) << 20;
constexpr int kMaxDevices = 64;
__device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];
void* g_scratch_ptr[kMaxDevices] = {};
std::mutex g_scratch_mu;

int scratch_of_current_device(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(CRBM_EUNSUPPORTED, "device %d is beyond the %d the library tracks", dev,
                                                   kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return fail(CRBM_EHIP, "hipGetSymbolAddress of the scratch array: %s", hipGetErrorString(e));
        }
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return CRBM_OK;
}
}  // namespace

extern "C" {

int crbm_fidelity_grad_noalloc(int n_visible, int n_hidden, const int8_t* samples, const void* T, const void* R,
                               long n, void* grad_out, double* loss_out, hipStream_t stream) {
    if (n_visible < 1 || n_hidden < 1) return fail(CRBM_EINVAL, "n_visible and n_hidden must be >= 1");
    if (n_visible > kMaxN || n_hidden > kMaxM)
        return fail(CRBM_EUNSUPPORTED, "N = %d, M = %d exceed the limits %d, %d", n_visible, n_hidden, kMaxN, kMaxM);
    if (!samples || !T || !R) return fail(CRBM_EINVAL, "samples, tanh_theta and R must be non-NULL");
    if (!grad_out && !loss_out) return fail(CRBM_EINVAL, "at least one of grad_out and loss_out must be non-NULL");
    if (n < 1) return fail(CRBM_EINVAL, "n_samples must be >= 1");
    const size_t need = fidelity_grad_scratch_bytes(n_visible, n_hidden, n);
    if (grad_out && need > kNoallocScratchBytes)
        return fail(CRBM_ENOMEM, "N = %d, M = %d, n = %ld need %zu bytes of scratch; the static scratch holds %zu",
                    n_visible, n_hidden, n, need, kNoallocScratchBytes);
    void* scr = nullptr;
    if (int rc = scratch_of_current_device(&scr)) return rc;
    GradArgs A{};
    A.N = n_visible; A.M = n_hidden; A.P = n_visible + n_hidden + n_visible * n_hidden;
    A.samples = samples;
    A.T = static_cast<const float2*>(T);
    A.R = static_cast<const float2*>(R);
    A.n = n;
    A.grad = static_cast<double2*>(grad_out);
    A.loss = loss_out;
    hipError_t e = launch_fidelity_grad_scratch(A, scr, current_cus(), stream);
    return e == hipSuccess ? CRBM_OK : hip_fail(e, "fidelity_grad_noalloc launch");
}

int crbm_moment_matrices(crbm_plan p, const crbm_rbm* gs, const void* t_params, const double* betas, int n_max,
                         const double* q, const int8_t* samples, const double* weights, long n, void* G_out,
                         void* H_out, hipStream_t stream) {
    if (check_plan(p)) return CRBM_EINVAL;
    if (int rc = check_rbm(p, gs, "psi_gs")) return rc;
    if (n_max < 0) return fail(CRBM_EINVAL, "n_max must be >= 0");
    if (n_max + 1 > kMaxBasis) return fail(CRBM_EUNSUPPORTED, "K = n_max + 1 = %d exceeds %d", n_max + 1, kMaxBasis);
    if (n_max > 0 && (!t_params || !betas)) return fail(CRBM_EINVAL, "t_params and betas must be non-NULL");
    if (!q) return fail(CRBM_EINVAL, "q is NULL");
    if (!samples || !G_out || !H_out) return fail(CRBM_EINVAL, "samples, G_out and H_out must be non-NULL");
    if (n < 1) return fail(CRBM_EINVAL, "n_samples must be >= 1");
    if (n > p->max_samples) return fail(CRBM_ENOMEM, "n_samples = %ld exceeds the plan's max_samples = %ld", n,
                                        p->max_samples);
    if (int rc = set_device(p)) return rc;
    const int K = n_max + 1;
    const size_t col_bytes = (size_t)K * (size_t)n * sizeof(float2);
    const char* fl = "CRBM_PLAN_BASIS";
    int rc = p->need(crbm_plan_s::GB_BASIS, col_bytes, fl);
    rc = rc ? rc : p->need(crbm_plan_s::GB_HBASIS, col_bytes, fl);
    rc = rc ? rc : p->need(crbm_plan_s::GB_ELOC, (size_t)n * sizeof(float2), fl);
    rc = rc ? rc : p->need(crbm_plan_s::GB_GRAM, (size_t)gram_partial_len(K) * sizeof(double2), fl);
    if (rc) return rc;
    float2* Bm = static_cast<float2*>(p->grow_ptr[crbm_plan_s::GB_BASIS]);
    float2* HBm = static_cast<float2*>(p->grow_ptr[crbm_plan_s::GB_HBASIS]);
    float2* loc = static_cast<float2*>(p->grow_ptr[crbm_plan_s::GB_ELOC]);
    double2* part = static_cast<double2*>(p->grow_ptr[crbm_plan_s::GB_GRAM]);
    const Geometry g = p->geometry();
    const RbmView vg = view(gs);
    const long P = p->P;
    const float2* tp = static_cast<const float2*>(t_params);

    // order 0: B_0 = f_q, HB_0 = (H S^z_q psi_gs)/psi_gs
    p->prof.begin(PROF_THETA, stream);
    hipError_t e = launch_theta(samples, n, p->N, p->M, vg.b, vg.W, p->theta[0], p->wplanes, stream);
    p->prof.end(stream);
    if (e == hipSuccess) e = launch_fq_chunk(g, samples, n, q, 1, p->momF, stream);
    LocalArgs A{};
    A.g = g;
    A.samples = samples;
    A.n_samples = n;
    A.eloc_out = loc;
    A.fit = vg;
    A.psn = vg;
    A.cheb_mode = 1;
    A.order = 0;
    A.W_scale = 1.0;
    A.q0 = q[0];
    A.q1 = p->lat.kind == CRBM_LATTICE_CHAIN ? 0.0 : q[1];
    if (e == hipSuccess) {
        p->prof.begin(PROF_LOCAL, stream);
        e = launch_local_core(A, p->theta[0], p->theta[0], nullptr, stream);
        p->prof.end(stream);
    }
    if (e == hipSuccess) e = launch_basis_pack(n, p->momF, loc, 0, Bm, HBm, stream);
    if (e == hipSuccess && n_max > 0) {
        p->prof.begin(PROF_MOMENT, stream);
        e = launch_lc_sums(samples, n, p->N, p->M, vg.a, vg.b, vg.W, p->wplanes, p->theta[2], nullptr, nullptr,
                           nullptr, p->lcLg, stream);
        p->prof.end(stream);
    }
    // orders 1..n_max: B_t = beta_t t~_t/psi_gs, HB_t = B_t E_loc[t~_t]
    for (int t = 1; t <= n_max && e == hipSuccess; ++t) {
        const float2* at = tp + (long)(t - 1) * P;
        RbmView vt;
        vt.a = at;
        vt.b = at + p->N;
        vt.W = at + p->N + p->M;
        p->prof.begin(PROF_THETA, stream);
        e = launch_theta(samples, n, p->N, p->M, vt.b, vt.W, p->theta[1], p->wplanes, stream);
        p->prof.end(stream);
        LocalArgs At{};
        At.g = g;
        At.samples = samples;
        At.n_samples = n;
        At.eloc_out = loc;
        At.fit = vt;
        if (e == hipSuccess) {
            p->prof.begin(PROF_LOCAL, stream);
            e = launch_local_core(At, p->theta[1], nullptr, nullptr, stream);
            p->prof.end(stream);
        }
        if (e == hipSuccess) {
            p->prof.begin(PROF_MOMENT, stream);
            e = launch_lc_sums(samples, n, p->N, p->M, at, vt.b, vt.W, p->wplanes, p->theta[2], p->lcLg,
                               reinterpret_cast<const double2*>(betas) + (t - 1), p->momB, nullptr, stream);
            p->prof.end(stream);
        }
        if (e == hipSuccess) e = launch_basis_pack(n, p->momB, loc, 1, Bm + (long)t * n, HBm + (long)t * n, stream);
    }
    if (e == hipSuccess) {
        p->prof.begin(PROF_GRAM, stream);
        e = launch_gram2(K, n, Bm, HBm, weights, 1.0 / (double)n, part, static_cast<double2*>(G_out),
                         static_cast<double2*>(H_out), 0, stream);
        p->prof.end(stream);
    }
    return e == hipSuccess ? CRBM_OK : hip_fail(e, "moment_matrices launch");
}

int crbm_sym_matrices(crbm_plan p, const crbm_rbm* gs, const void* t_params, const double* betas, int n_max,
                      int rotations, const int8_t* samples, const double* weights, long n, void* G_out, void* H_out,
                      hipStream_t stream) {
    if (check_plan(p)) return CRBM_EINVAL;
    if (int rc = check_rbm(p, gs, "psi_gs")) return rc;
    if (n_max < 0) return fail(CRBM_EINVAL, "n_max must be >= 0");
    if (n_max + 1 > kMaxBasis) return fail(CRBM_EUNSUPPORTED, "K = n_max + 1 = %d exceeds %d", n_max + 1, kMaxBasis);
    if (n_max > 0 && (!t_params || !betas)) return fail(CRBM_EINVAL, "t_params and betas must be non-NULL");
    if (!samples || !G_out || !H_out) return fail(CRBM_EINVAL, "samples, G_out and H_out must be non-NULL");
    if (rotations != 0 && rotations != 1) return fail(CRBM_EINVAL, "rotations must be 0 or 1");
    if (rotations && (p->lat.kind != CRBM_LATTICE_SQUARE || p->lat.Lx != p->lat.Ly))
        return fail(CRBM_EINVAL, "rotations need a square L x L lattice");
    if (n < 1) return fail(CRBM_EINVAL, "n_samples must be >= 1");
    const int N = p->N, M = p->M, K = n_max + 1;
    const int nrot = rotations ? 4 : 1;
    const long ng = (long)N * nrot;
    if (ng > p->max_samples)
        return fail(CRBM_EUNSUPPORTED, "the plan's max_samples = %ld is below the %ld images of one sample",
                    p->max_samples, ng);
    if (int rc = set_device(p)) return rc;
    const long cmax = p->max_samples / ng;                  // samples per chunk
    const long rows_max = cmax * ng;
    const size_t colb = (size_t)K * (size_t)rows_max * sizeof(float2);
    const char* fl = "CRBM_PLAN_SYM_BASIS";
    int rc = p->need(crbm_plan_s::GB_BASIS, colb, fl);
    rc = rc ? rc : p->need(crbm_plan_s::GB_HBASIS, colb, fl);
    rc = rc ? rc : p->need(crbm_plan_s::GB_SYMBT, colb, fl);
    rc = rc ? rc : p->need(crbm_plan_s::GB_SYMHBT, colb, fl);
    rc = rc ? rc : p->need(crbm_plan_s::GB_SYMIMG, (size_t)rows_max * N, fl);
    rc = rc ? rc : p->need(crbm_plan_s::GB_SYMLT, (size_t)rows_max * sizeof(float2), fl);
    rc = rc ? rc : p->need(crbm_plan_s::GB_ELOC, (size_t)rows_max * sizeof(float2), fl);
    rc = rc ? rc : p->need(crbm_plan_s::GB_SYMLG, (size_t)cmax * sizeof(float2), fl);
    rc = rc ? rc : p->need(crbm_plan_s::GB_GRAM, (size_t)gram_partial_len(K) * sizeof(double2), fl);
    if (rc) return rc;
    float2* Bm = static_cast<float2*>(p->grow_ptr[crbm_plan_s::GB_BASIS]);
    float2* HBm = static_cast<float2*>(p->grow_ptr[crbm_plan_s::GB_HBASIS]);
    float2* Bt = static_cast<float2*>(p->grow_ptr[crbm_plan_s::GB_SYMBT]);
    float2* HBt = static_cast<float2*>(p->grow_ptr[crbm_plan_s::GB_SYMHBT]);
    int8_t* img = static_cast<int8_t*>(p->grow_ptr[crbm_plan_s::GB_SYMIMG]);
    float2* lt = static_cast<float2*>(p->grow_ptr[crbm_plan_s::GB_SYMLT]);
    float2* el = static_cast<float2*>(p->grow_ptr[crbm_plan_s::GB_ELOC]);
    float2* lg = static_cast<float2*>(p->grow_ptr[crbm_plan_s::GB_SYMLG]);
    double2* part = static_cast<double2*>(p->grow_ptr[crbm_plan_s::GB_GRAM]);
    double2* G = static_cast<double2*>(G_out);
    double2* H = static_cast<double2*>(H_out);
    const Geometry geo = p->geometry();
    const RbmView vg = view(gs);
    const long P = p->P;
    const float2* tp = static_cast<const float2*>(t_params);
    const int Ly = p->lat.kind == CRBM_LATTICE_CHAIN ? 1 : p->lat.Ly;
    hipError_t e = hipSuccess;
    auto theta = [&](const int8_t* sig, long rows, const RbmView& v, float2* out) {
        p->prof.begin(PROF_THETA, stream);
        hipError_t r = launch_theta(sig, rows, N, M, v.b, v.W, out, p->wplanes, stream);
        p->prof.end(stream);
        return r;
    };
    auto local = [&](const LocalArgs& A, const float2* th) {
        p->prof.begin(PROF_LOCAL, stream);
        hipError_t r = launch_local_core(A, th, th, nullptr, stream);
        p->prof.end(stream);
        return r;
    };
    for (long s0 = 0; s0 < n && e == hipSuccess; s0 += cmax) {
        const long c = (n - s0) < cmax ? (n - s0) : cmax;
        const long rows = c * ng;
        const int8_t* sig = samples + s0 * N;
        // log psi_gs of the chunk's samples
        e = theta(sig, c, vg, p->theta[2]);
        LocalArgs A0{};
        A0.g = geo; A0.fit = vg; A0.samples = sig; A0.n_samples = c; A0.logpsi_out = lg;
        if (e == hipSuccess) e = local(A0, p->theta[2]);
        // the images of every sample under the group
        if (e == hipSuccess) e = launch_sym_images(sig, c, N, p->lat.kind, p->lat.Lx, Ly, nrot, img, stream);
        // order 0: t_000 = S^z_0 psi_gs on the images
        if (e == hipSuccess) e = theta(img, rows, vg, p->theta[0]);
        LocalArgs A1{};
        A1.g = geo; A1.fit = vg; A1.psn = vg; A1.cheb_mode = 1; A1.local_op = 1; A1.order = 0; A1.W_scale = 1.0;
        A1.samples = img; A1.n_samples = rows; A1.logpsi_out = lt; A1.eloc_out = el;
        if (e == hipSuccess) e = local(A1, p->theta[0]);
        if (e == hipSuccess) e = launch_sym_combine(rows, (int)ng, N, img, 1, lt, el, lg, nullptr, Bm, HBm, stream);
        for (int t = 1; t <= n_max && e == hipSuccess; ++t) {
            const float2* at = tp + (long)(t - 1) * P;
            RbmView vt;
            vt.a = at; vt.b = at + N; vt.W = at + N + M;
            e = theta(img, rows, vt, p->theta[1]);
            LocalArgs At{};
            At.g = geo; At.fit = vt; At.samples = img; At.n_samples = rows; At.logpsi_out = lt; At.eloc_out = el;
            if (e == hipSuccess) e = local(At, p->theta[1]);
            if (e == hipSuccess)
                e = launch_sym_combine(rows, (int)ng, N, img, 0, lt, el, lg,
                                       reinterpret_cast<const double2*>(betas) + (t - 1), Bm + (long)t * rows,
                                       HBm + (long)t * rows, stream);
        }
        // momentum projection for all N momenta, then G^(k), H^(k) accumulated over chunks
        if (e == hipSuccess) e = launch_sym_dft(c, K, N, p->lat.kind, p->lat.Lx, Ly, nrot, Bm, HBm, Bt, HBt, stream);
        p->prof.begin(PROF_GRAM, stream);
        for (int kk = 0; kk < N && e == hipSuccess; ++kk)
            e = launch_gram2(K, c, Bt + (long)kk * K * c, HBt + (long)kk * K * c, weights ? weights + s0 : nullptr,
                             1.0 / (double)n, part, G + (long)kk * K * K, H + (long)kk * K * K, s0 > 0, stream);
        p->prof.end(stream);
    }
    return e == hipSuccess ? CRBM_OK : hip_fail(e, "sym_matrices launch");
}

int crbm_corrected_moments(crbm_plan p, const void* G, const void* H, int K, double E_c, double W_scale, int n_out,
                           double* mu_out, double* info_out, hipStream_t stream) {
    if (check_plan(p)) return CRBM_EINVAL;
    if (!G || !H || !mu_out || !info_out) return fail(CRBM_EINVAL, "G, H, mu_out and info_out must be non-NULL");
    if (K < 1 || K > kMaxBasis) return fail(CRBM_EINVAL, "K must be in [1, %d] (got %d)", kMaxBasis, K);
    if (n_out < 1) return fail(CRBM_EINVAL, "n_out must be >= 1");
    if (!(W_scale != 0.0) || !(W_scale - W_scale == 0.0) || !(E_c - E_c == 0.0))
        return fail(CRBM_EINVAL, "E_c must be finite and W_scale finite and non-zero");
    if (int rc = set_device(p)) return rc;
    hipError_t e = launch_correct(K, static_cast<const double2*>(G), static_cast<const double2*>(H), E_c, W_scale,
                                  n_out, static_cast<double2*>(p->grow_ptr[crbm_plan_s::GB_SMALL]), mu_out, info_out,
                                  stream);
    return e == hipSuccess ? CRBM_OK : hip_fail(e, "corrected_moments launch");
}

int crbm_lanczos(crbm_plan p, const void* G, const void* H, int K, int n_steps, double* a_out, double* b2_out,
                 double* info_out, hipStream_t stream) {
    if (check_plan(p)) return CRBM_EINVAL;
    if (!G || !H || !a_out || !b2_out || !info_out)
        return fail(CRBM_EINVAL, "G, H, a_out, b2_out and info_out must be non-NULL");
    if (K < 1 || K > kMaxBasis) return fail(CRBM_EINVAL, "K must be in [1, %d] (got %d)", kMaxBasis, K);
    if (n_steps < 1) return fail(CRBM_EINVAL, "n_steps must be >= 1");
    if (int rc = set_device(p)) return rc;
    hipError_t e = launch_lanczos(K, static_cast<const double2*>(G), static_cast<const double2*>(H), n_steps,
                                  static_cast<double2*>(p->grow_ptr[crbm_plan_s::GB_SMALL]), a_out, b2_out, info_out,
                                  stream);
    return e == hipSuccess ? CRBM_OK : hip_fail(e, "lanczos launch");
}

int crbm_spectrum_kpm(const double* mu, int n_mom, int jackson, double E0, double E_c, double W_scale,
                      const double* omega, int n_omega, double* A_out, hipStream_t stream) {
    if (!mu || !omega || !A_out) return fail(CRBM_EINVAL, "mu, omega and A_out must be non-NULL");
    if (n_mom < 1) return fail(CRBM_EINVAL, "n_mom must be >= 1");
    if (n_omega < 0) return fail(CRBM_EINVAL, "n_omega must be >= 0");
    if (!(W_scale != 0.0) || !(W_scale - W_scale == 0.0)) return fail(CRBM_EINVAL, "W_scale must be finite and non-zero");
    if (n_omega == 0) return CRBM_OK;
    hipError_t e = launch_spec_kpm(mu, n_mom, jackson != 0, E0, E_c, W_scale, omega, n_omega, A_out, stream);
    return e == hipSuccess ? CRBM_OK : hip_fail(e, "spectrum_kpm launch");
}

int crbm_spectrum_cf(const double* a, const double* b2, int m, double E0, double eta, const double* omega, int n_omega,
                     double* A_out, hipStream_t stream) {
    if (!a || !b2 || !omega || !A_out) return fail(CRBM_EINVAL, "a, b2, omega and A_out must be non-NULL");
    if (m < 1) return fail(CRBM_EINVAL, "m must be >= 1");
    if (n_omega < 0) return fail(CRBM_EINVAL, "n_omega must be >= 0");
    if (!(eta > 0.0)) return fail(CRBM_EINVAL, "eta must be > 0");
    if (n_omega == 0) return CRBM_OK;
    hipError_t e = launch_spec_cf(a, b2, m, E0, eta, omega, n_omega, A_out, stream);
    return e == hipSuccess ? CRBM_OK : hip_fail(e, "spectrum_cf launch");
}

int crbm_probe_mfma(double* tflops_out, hipStream_t stream) {
    if (!tflops_out) return fail(CRBM_EINVAL, "tflops_out is NULL");
    const int blocks = 2 * current_cus(), iters = 20000;
    float* out = nullptr;
    hipError_t e = hipMalloc(&out, (size_t)blocks * 256 * sizeof(float));
    if (e != hipSuccess) { (void)hipGetLastError(); return fail(CRBM_ENOMEM, "probe buffer: %s", hipGetErrorString(e)); }
    auto launch = [&]() { return launch_probe_mfma(blocks, iters, out, stream); };
    double ms = timed_ms(stream, launch);          // the first launch brings the clocks up
    if (ms > 0) ms = timed_ms(stream, launch);
    (void)hipFree(out);
    if (!(ms > 0)) return fail(CRBM_EHIP, "matrix-core probe failed");
    *tflops_out = (double)blocks * 4 * iters * 8 * 32768.0 / (ms * 1e-3) / 1e12;
    return CRBM_OK;
}

int crbm_probe_logcosh(double* evals_out, hipStream_t stream) {
    if (!evals_out) return fail(CRBM_EINVAL, "evals_out is NULL");
    const int blocks = 8 * current_cus(), iters = 4000;
    float* out = nullptr;
    hipError_t e = hipMalloc(&out, (size_t)blocks * 256 * sizeof(float));
    if (e != hipSuccess) { (void)hipGetLastError(); return fail(CRBM_ENOMEM, "probe buffer: %s", hipGetErrorString(e)); }
    auto launch = [&]() { return launch_probe_logcosh(blocks, iters, out, stream); };
    double ms = timed_ms(stream, launch);
    if (ms > 0) ms = timed_ms(stream, launch);
    (void)hipFree(out);
    if (!(ms > 0)) return fail(CRBM_EHIP, "log-cosh probe failed");
    *evals_out = (double)blocks * 256 * iters * 8 / (ms * 1e-3);
    return CRBM_OK;
}

int crbm_probe_gather(int n_rows, int row_elems, double* gbs_out, hipStream_t stream) {
    if (!gbs_out) return fail(CRBM_EINVAL, "gbs_out is NULL");
    if (n_rows < 1 || row_elems < 1 || (long)n_rows * row_elems > (1L << 24))
        return fail(CRBM_EINVAL, "need n_rows, row_elems >= 1 and a table of at most 2^24 entries");
    const int blocks = 8 * current_cus(), iters = 2000;
    float2* tab = nullptr;
    float* out = nullptr;
    hipError_t e = hipMalloc(&tab, (size_t)n_rows * row_elems * sizeof(float2));
    if (e == hipSuccess) e = hipMalloc(&out, (size_t)blocks * 256 * sizeof(float));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        if (tab) (void)hipFree(tab);
        return fail(CRBM_ENOMEM, "probe buffers: %s", hipGetErrorString(e));
    }
    auto launch = [&]() { return launch_probe_gather(blocks, tab, n_rows, row_elems, iters, out, stream); };
    e = hipMemsetAsync(tab, 0, (size_t)n_rows * row_elems * sizeof(float2), stream);
    double ms = e == hipSuccess ? timed_ms(stream, launch) : -1.0;
    if (ms > 0) ms = timed_ms(stream, launch);
    (void)hipFree(tab);
    (void)hipFree(out);
    if (!(ms > 0)) return fail(CRBM_EHIP, "gather probe failed");
    *gbs_out = (double)blocks * 4 * iters * row_elems * sizeof(float2) / (ms * 1e-3) / 1e9;
    return CRBM_OK;
}

int crbm_probe_hbm(size_t bytes, double* gbs_out, hipStream_t stream) {
    if (!gbs_out) return fail(CRBM_EINVAL, "gbs_out is NULL");
    if (bytes < (1u << 20)) return fail(CRBM_EINVAL, "bytes must be >= 1 MiB");
    const long n16 = (long)(bytes / 16);
    void *a = nullptr, *b = nullptr;
    hipError_t e = hipMalloc(&a, (size_t)n16 * 16);
    if (e == hipSuccess) e = hipMalloc(&b, (size_t)n16 * 16);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        if (a) (void)hipFree(a);
        return fail(CRBM_ENOMEM, "probe buffers: %s", hipGetErrorString(e));
    }
    const int blocks = 8 * current_cus();
    auto launch = [&]() { return launch_probe_copy(blocks, a, b, n16, stream); };
    e = hipMemsetAsync(a, 1, (size_t)n16 * 16, stream);
    double ms = e == hipSuccess ? timed_ms(stream, launch) : -1.0;
    if (ms > 0) ms = timed_ms(stream, launch);
    (void)hipFree(a);
    (void)hipFree(b);
    if (!(ms > 0)) return fail(CRBM_EHIP, "HBM probe failed");
    *gbs_out = 2.0 * (double)n16 * 16 / (ms * 1e-3) / 1e9;
    return CRBM_OK;
}

static int batched_args(crbm_plan p, const crbm_rbm* gs, const void* t_params, const double* betas, const double* q,
                        const int64_t* offsets, int n_inst, int64_t total, int n_burn, int n_sweeps, int proposal,
                        uint64_t seed, BatchedArgs& A) {
    if (check_plan(p)) return CRBM_EINVAL;
    if (int rc = check_rbm(p, gs, "psi_gs")) return rc;
    if (!t_params || !betas || !q || !offsets) return fail(CRBM_EINVAL, "t_params, betas, q and chain_offsets must be non-NULL");
    if (n_inst < 1) return fail(CRBM_EINVAL, "n_inst must be >= 1");
    if (total < 0 || total > p->max_samples)
        return fail(CRBM_ENOMEM, "total_chains = %lld must be in [0, max_samples = %ld]", (long long)total, p->max_samples);
    if (n_burn < 0 || n_sweeps < 1) return fail(CRBM_EINVAL, "need n_burn >= 0 and n_sweeps >= 1");
    if ((int64_t)(n_burn + (int64_t)n_sweeps) * p->N > INT32_MAX)
        return fail(CRBM_EINVAL, "(n_burn + n_sweeps) * N = %lld proposals per chain exceed 2^31 - 1",
                    (long long)((n_burn + (int64_t)n_sweeps) * p->N));
    if (proposal != CRBM_PROPOSAL_FLIP && proposal != CRBM_PROPOSAL_EXCHANGE)
        return fail(CRBM_EINVAL, "unknown proposal %d", proposal);
    if (p->N % 2) return fail(CRBM_EINVAL, "the S^z = 0 chain starts need an even number of sites");
    if (int rc = set_device(p)) return rc;
    A.N = p->N; A.M = p->M; A.P = (int)p->P; A.kind = p->lat.kind; A.Lx = p->lat.Lx;
    A.gs = view(gs);
    A.t_params = static_cast<const float2*>(t_params);
    A.betas = reinterpret_cast<const double2*>(betas);
    A.q = q;
    A.offsets = offsets;
    A.n_inst = n_inst;
    A.total = total;
    A.n_burn = n_burn;
    A.n_sweeps = n_sweeps;
    A.proposal = proposal;
    A.seed = seed;
    A.counter = p->bcounter;
    A.partial = p->bpartial;
    return CRBM_OK;
}

int crbm_batched_moments(crbm_plan p, const crbm_rbm* gs, const void* t_params, const double* betas, const double* q,
                         const int64_t* offsets, int n_inst, int64_t total, int n_burn, int n_sweeps, int proposal,
                         uint64_t seed, void* mu_out, uint32_t* trace, hipStream_t stream) {
    BatchedArgs A{};
    if (int rc = batched_args(p, gs, t_params, betas, q, offsets, n_inst, total, n_burn, n_sweeps, proposal, seed, A))
        return rc;
    if (!mu_out) return fail(CRBM_EINVAL, "mu_out is NULL");
    A.trace = trace;
    A.trace_words = (int)(((long)(n_burn + n_sweeps) * p->N + 31) / 32);
    if (p->prof.on) {
        // every row is rewritten or cleared, so rows of an earlier, larger grid do not linger
        hipError_t ec = launch_clear_u64(p->bclocks, (long)2 * CRBM_MAX_CLOCK_WAVES, stream);
        if (ec != hipSuccess) return hip_fail(ec, "batched_moments clock clear");
        A.clocks = p->bclocks;
    }
    p->prof.begin(PROF_BATCHED, stream);
    hipError_t e = launch_batched(A, p->b_blocks, p->b_waves, p->b_lanes, static_cast<double2*>(mu_out), stream);
    p->prof.end(stream);
    return e == hipSuccess ? CRBM_OK : hip_fail(e, "batched_moments launch");
}

int crbm_batched_autotune(crbm_plan p, const crbm_rbm* gs, const void* t_params, const double* betas, const double* q,
                          const int64_t* offsets, int n_inst, int64_t total, int n_probe, int proposal, uint64_t seed,
                          void* mu_scratch, int* waves_out, int* blocks_out, int* lanes_out, double* ms_out,
                          hipStream_t stream) {
    BatchedArgs A{};
    if (int rc = batched_args(p, gs, t_params, betas, q, offsets, n_inst, total, 0, n_probe, proposal, seed, A))
        return rc;
    if (!mu_scratch) return fail(CRBM_EINVAL, "mu_scratch is NULL");
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return fail(CRBM_EHIP, "hipEventCreate");
    double best = 1e300;
    int bw = p->b_waves, bb = p->b_blocks, bl = p->b_lanes;
    const int waves[4] = {1, 2, 4, 8}, per_cu[4] = {1, 2, 4, 8}, lanes[3] = {64, 32, 16};
    for (int li = 0; li < 3; ++li) {
        if (!batched_lanes_ok(lanes[li], p->M)) continue;
        for (int wi = 0; wi < 4; ++wi)
            for (int ci = 0; ci < 4; ++ci) {
                const int blocks = per_cu[ci] * p->n_cu;
                hipError_t r = hipEventRecord(e0, stream);
                if (r == hipSuccess)
                    r = launch_batched(A, blocks, waves[wi], lanes[li], static_cast<double2*>(mu_scratch), stream);
                if (r == hipSuccess) r = hipEventRecord(e1, stream);
                if (r == hipSuccess) r = hipEventSynchronize(e1);
                float ms = 0.f;
                if (r == hipSuccess) r = hipEventElapsedTime(&ms, e0, e1);
                if (r != hipSuccess) {
                    (void)hipEventDestroy(e0);
                    (void)hipEventDestroy(e1);
                    return hip_fail(r, "batched autotune");
                }
                if (ms < best) { best = ms; bw = waves[wi]; bb = blocks; bl = lanes[li]; }
            }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    p->b_waves = bw;
    p->b_blocks = bb;
    p->b_lanes = bl;
    if (waves_out) *waves_out = bw;
    if (blocks_out) *blocks_out = bb;
    if (lanes_out) *lanes_out = bl;
    if (ms_out) *ms_out = best;
    return CRBM_OK;
}

int crbm_plan_set_sbuild_tile(crbm_plan p, int k_tile) {
    if (check_plan(p)) return CRBM_EINVAL;
    if (k_tile != 64 && k_tile != 128) return fail(CRBM_EINVAL, "k_tile must be 64 or 128, got %d", k_tile);
    p->w.sb_kt = k_tile;
    return CRBM_OK;
}

int crbm_sbuild_autotune(crbm_plan p, const int8_t* samples, const void* tanh_theta, long n, int* k_tile_out,
                         double* best_ms, hipStream_t stream) {
    if (check_plan(p)) return CRBM_EINVAL;
    if (!p->w.S || !p->w.pack) return fail(CRBM_EINVAL, "the plan holds no dense S (create it with CRBM_PLAN_DENSE_S)");
    if (!samples || !tanh_theta) return fail(CRBM_EINVAL, "samples and tanh_theta must be non-NULL");
    if (n < 1 || n > p->max_samples) return fail(CRBM_ENOMEM, "n = %ld must be in [1, max_samples = %ld]", n, p->max_samples);
    if (int rc = set_device(p)) return rc;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return fail(CRBM_EHIP, "hipEventCreate");
    const int nsplit = p->w.spart ? sbuild_splits((int)p->N, (int)p->M, n, p->w.n_cu, p->w.nsplit_max) : 1;
    const int nsb = sbuild_border_splits((int)p->N, (int)p->M, n, p->w.n_cu, p->w.nsb_max);
    Profiler off;
    double best = 1e300;
    int bk = p->w.sb_kt;
    const int tiles[2] = {128, 64};
    for (int ti = 0; ti < 2; ++ti) {
        float ms = 0.f;
        hipError_t r = hipEventRecord(e0, stream);
        if (r == hipSuccess)
            r = launch_sbuild_mfma((int)p->N, (int)p->M, p->P, samples, static_cast<const float2*>(tanh_theta), n,
                                   p->w.Om, p->w.Om, p->w.S, CRBM_PREC_BF16, tiles[ti], p->w.pack, p->w.pack_bytes,
                                   p->w.sb_order, p->w.sb_order_len,
                                   p->w.spart, nsplit, p->w.bx, p->w.bx_part, nsb, &off, stream);
        if (r == hipSuccess) r = hipEventRecord(e1, stream);
        if (r == hipSuccess) r = hipEventSynchronize(e1);
        if (r == hipSuccess) r = hipEventElapsedTime(&ms, e0, e1);
        if (r != hipSuccess) {
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            return hip_fail(r, "sbuild autotune");
        }
        if (ms < best) { best = ms; bk = tiles[ti]; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    p->w.sb_kt = bk;
    if (k_tile_out) *k_tile_out = bk;
    if (best_ms) *best_ms = best;
    return CRBM_OK;
}

int crbm_batched_set_shape(crbm_plan p, int waves_per_block, int blocks, int lanes_per_chain) {
    if (check_plan(p)) return CRBM_EINVAL;
    if (waves_per_block < 1 || waves_per_block > 8) return fail(CRBM_EINVAL, "waves_per_block must be in [1, 8]");
    if (blocks < 1) return fail(CRBM_EINVAL, "blocks must be >= 1");
    if (!batched_lanes_ok(lanes_per_chain, (int)p->M))
        return fail(CRBM_EUNSUPPORTED, "lanes_per_chain = %d is not 64, 32 (M <= 256) or 16 (M <= 128) for M = %ld",
                    lanes_per_chain, p->M);
    p->b_waves = waves_per_block;
    p->b_blocks = blocks;
    p->b_lanes = lanes_per_chain;
    return CRBM_OK;
}

int crbm_batched_lds_rows(crbm_plan p, int proposal, int waves_per_block, int* uses) {
    if (check_plan(p)) return CRBM_EINVAL;
    if (!uses) return fail(CRBM_EINVAL, "uses is NULL");
    if (proposal != CRBM_PROPOSAL_FLIP && proposal != CRBM_PROPOSAL_EXCHANGE) return fail(CRBM_EINVAL, "unknown proposal %d", proposal);
    if (waves_per_block < 1 || waves_per_block > 8) return fail(CRBM_EINVAL, "waves_per_block must be in [1, 8]");
    if (int rc = set_device(p)) return rc;
    *uses = batched_lds_rows((int)p->N, (int)p->M, proposal, waves_per_block) ? 1 : 0;
    return CRBM_OK;
}

}  // extern "C"
