// C ABI of the Wilson library: context, field conversion, operators, BLAS and
// the conjugate-gradient driver.  All arithmetic happens in the kernels of
// wl_dslash.hip and wl_blas.hip; this file validates arguments, owns device
// memory and enqueues launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <array>
#include <vector>

#include "wilson.h"
#include "wl_blas.h"
#include "wl_dslash.h"
#include "wl_ptc.h"
#include "wl_access.h"
#include "wl_halo.h"

using namespace wl;

// ------------------------------------------------------------------ errors
static thread_local std::string g_err;

static wl_status fail(wl_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define HIP_TRY(call)                                                                            \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess) return fail(WL_ERR_HIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

// ------------------------------------------------------------------ context
namespace {
enum Slot {
    S_TMP_OP = 0,  // odd temporary of wl_dirac_apply
    S_R, S_P, S_Q, S_S, S_TMP,           // solver fields in the inner precision
    S_RHI, S_THI, S_TMPHI,               // FP64 fields for true residuals
    S_XLO,                               // FP32 accumulator of x steps between refreshes (mixed precision)
    S_PARTIALS, S_SCAL, S_BNORM, S_FLAG,
    S_PTC_H, S_PTC_GH, S_PTC_O, S_PTC_GO, S_PTC_PART, S_PTC_E2,       // PTC workspace
    S_GCR_R, S_GCR_X, S_GCR_Z, S_GCR_W, S_GCR_TMP, S_GCR_RHS,          // FGCR workspace
    S_PCG,                                                             // preconditioned CGNR workspace
    S_FACE,                                                            // t-face send / receive buffers
    S_NSLOTS
};
}

struct wl_ctx {
    int dims[4];
    double phases[8];
    long V, Vh;
    int device;
    Geom g;
    void *gauge[5][2] = {};  // [prec][recon == 12]
    size_t slab[5][2] = {};
    void *buf[S_NSLOTS] = {};
    size_t buf_bytes[S_NSLOTS] = {};
    void *host_pinned = nullptr;
    size_t host_pinned_bytes = 0;
    LaunchCfg cfg[5];  // hopping-kernel launch configuration per storage precision
    // kernel timing
    bool timing = false;
    int timing_stride = 1;  // record every timing_stride-th hopping launch
    unsigned long timing_seq = 0;
    struct TimedLaunch {
        int key;
        hipEvent_t ev[2];
        int iter;   // CG iteration the launch belongs to (-1: none)
        int cycle;  // CG cycle serial number
    };
    int timing_iter = -1;
    int timing_cycle = 0;
    std::vector<TimedLaunch> timed;
    std::vector<hipEvent_t> event_pool;
    size_t pool_used = 0;
    bool capturing = false;  // no timing events inside a stream capture
    // hipGraph replay of one CG iteration (solver param use_graph)
    hipStream_t own_stream = nullptr;  // capture needs a stream other than the null stream
    hipEvent_t handoff[2] = {nullptr, nullptr};
    hipGraph_t cg_graph = nullptr;
    hipGraphExec_t cg_exec = nullptr;
    std::vector<uintptr_t> cg_graph_key;
    // bulk / boundary split: the stream the face exchange runs on, and its events
    hipStream_t comm_stream = nullptr;
    hipEvent_t halo_ev[2] = {nullptr, nullptr};
};

static int timing_key(int prec, int recon, int dagger, int epi) {
    return ((prec * 2 + (recon == 12 ? 1 : 0)) * 2 + (dagger ? 1 : 0)) * 8 + epi;
}

static bool prec_ok(int p) { return p >= WL_F64 && p <= WL_I16N; }
static bool recon_ok(int prec, int r) {
    if (r != 12 && r != 18) return false;
    if (prec >= WL_F16N && r != 12) return false;
    return true;
}

static size_t half_bytes(const wl_ctx *c, int prec, int nrhs) {
    return spinor_point_bytes(prec) * (size_t)padded(c->Vh * (long)nrhs);
}

static wl_status ensure_buf(wl_ctx *c, int slot, size_t bytes) {
    if (c->buf_bytes[slot] >= bytes) return WL_OK;
    if (c->buf[slot]) {
        HIP_TRY(hipDeviceSynchronize());
        HIP_TRY(hipFree(c->buf[slot]));
        c->buf[slot] = nullptr;
        c->buf_bytes[slot] = 0;
    }
    hipError_t e = hipMalloc(&c->buf[slot], bytes);
    if (e != hipSuccess) {
        c->buf[slot] = nullptr;
        (void)hipGetLastError();
        return fail(WL_ERR_NOMEM, "hipMalloc of %zu bytes failed: %s", bytes, hipGetErrorString(e));
    }
    c->buf_bytes[slot] = bytes;
    return WL_OK;
}

static wl_status ensure_pinned(wl_ctx *c, size_t bytes) {
    if (c->host_pinned_bytes >= bytes) return WL_OK;
    if (c->host_pinned) HIP_TRY(hipHostFree(c->host_pinned));
    c->host_pinned = nullptr;
    c->host_pinned_bytes = 0;
    HIP_TRY(hipHostMalloc(&c->host_pinned, bytes, hipHostMallocDefault));
    c->host_pinned_bytes = bytes;
    return WL_OK;
}

// ------------------------------------------------------------------ small kernels (layout conversion)
// canonical FP64 spinor <-> internal, one thread per internal point
template <int SP>
__global__ void __launch_bounds__(256) k_pack(Geom g, void *dst, size_t half_bytes, const double *src, int subset,
                                              int nrhs) {
    using T = typename SpinorIO<SP>::real;
    const int h = blockIdx.y;
    const long n = (long)g.vh * nrhs;
    const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= n) return;
    const int i = (int)(gid / nrhs), rhs = (int)(gid - (long)i * nrhs);
    const int par = subset == WL_FULL ? h : subset;
    long idx, nsite;
    if (subset == WL_FULL) {
        int c[4];
        eo_coords(g, i, par, c);
        idx = c[0] + (long)g.L[0] * (c[1] + (long)g.L[1] * (c[2] + (long)g.L[2] * c[3]));
        nsite = 2L * g.vh;
    } else {
        idx = i;
        nsite = g.vh;
    }
    const double *s = src + ((long)rhs * nsite + idx) * 24;
    cpx<T> v[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) v[k] = {(T)s[2 * k], (T)s[2 * k + 1]};
    SpinorIO<SP>::store((char *)dst + h * half_bytes, gid, v);
}

template <int SP>
__global__ void __launch_bounds__(256) k_unpack(Geom g, double *dst, const void *src, size_t half_bytes, int subset,
                                                int nrhs) {
    using T = typename SpinorIO<SP>::real;
    const int h = blockIdx.y;
    const long n = (long)g.vh * nrhs;
    const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= n) return;
    const int i = (int)(gid / nrhs), rhs = (int)(gid - (long)i * nrhs);
    const int par = subset == WL_FULL ? h : subset;
    long idx, nsite;
    if (subset == WL_FULL) {
        int c[4];
        eo_coords(g, i, par, c);
        idx = c[0] + (long)g.L[0] * (c[1] + (long)g.L[1] * (c[2] + (long)g.L[2] * c[3]));
        nsite = 2L * g.vh;
    } else {
        idx = i;
        nsite = g.vh;
    }
    cpx<T> v[12];
    SpinorIO<SP>::load((const char *)src + h * half_bytes, gid, v);
    double *d = dst + ((long)rhs * nsite + idx) * 24;
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        d[2 * k] = (double)v[k].re;
        d[2 * k + 1] = (double)v[k].im;
    }
}

// FP64 18-real internal links -> another link format, one thread per (slab, site)
template <int GP, int R>
__global__ void __launch_bounds__(256) k_link_convert(void *dst, size_t dslab, const void *src, size_t sslab,
                                                      int vh) {
    using T = typename LinkIO<GP, R>::real;
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int slab = blockIdx.y;
    if (i >= vh) return;
    cpx<double> u[9];
    LinkIO<WL_F64, 18>::load((const char *)src + slab * sslab, i, u);
    cpx<T> w[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) w[k] = {(T)u[k].re, (T)u[k].im};
    LinkIO<GP, R>::store((char *)dst + slab * dslab, i, w);
}

template <template <int> class K, typename... A>
static hipError_t launch_prec(int prec, dim3 grid, hipStream_t s, A... args) {
    switch (prec) {
    case WL_F64: hipLaunchKernelGGL(K<WL_F64>::fn, grid, dim3(256), 0, s, args...); break;
    case WL_F32: hipLaunchKernelGGL(K<WL_F32>::fn, grid, dim3(256), 0, s, args...); break;
    case WL_F16N: hipLaunchKernelGGL(K<WL_F16N>::fn, grid, dim3(256), 0, s, args...); break;
    case WL_BF16N: hipLaunchKernelGGL(K<WL_BF16N>::fn, grid, dim3(256), 0, s, args...); break;
    case WL_I16N: hipLaunchKernelGGL(K<WL_I16N>::fn, grid, dim3(256), 0, s, args...); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
template <int SP> struct PackK { static constexpr auto fn = k_pack<SP>; };
template <int SP> struct UnpackK { static constexpr auto fn = k_unpack<SP>; };

// ------------------------------------------------------------------ validation helpers
static wl_status check_field_args(const wl_ctx *c, int subset, int prec, int nrhs) {
    if (!c) return fail(WL_ERR_ARG, "null context");
    if (subset < WL_EVEN || subset > WL_FULL) return fail(WL_ERR_ARG, "bad subset %d", subset);
    if (!prec_ok(prec)) return fail(WL_ERR_ARG, "bad precision %d", prec);
    if (nrhs < 1 || nrhs > 64) return fail(WL_ERR_ARG, "nrhs %d outside [1, 64]", nrhs);
    return WL_OK;
}
static bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }
static bool overlap(const void *a, size_t na, const void *b, size_t nb) {
    const char *x = (const char *)a, *y = (const char *)b;
    return x < y + nb && y < x + na;
}

static wl_status get_links(wl_ctx *c, int prec, int recon, const void **ptr, size_t *slab);

// ------------------------------------------------------------------ context API
extern "C" const char *wl_last_error(void) { return g_err.c_str(); }
extern "C" const char *wl_version(void) { return "wilson-gfx950 0.1"; }

extern "C" wl_status wl_ctx_create(const int dims[4], const double phases[8], const double *gauge_host,
                                   wl_ctx **out) {
    g_err.clear();
    if (!dims || !phases || !gauge_host || !out) return fail(WL_ERR_ARG, "null argument");
    *out = nullptr;
    long V = 1;
    for (int m = 0; m < 4; ++m) {
        if (dims[m] < 2 || dims[m] % 2 || dims[m] > 4096)
            return fail(WL_ERR_DIMS, "extent %d of direction %d must be even and in [2, 4096]", dims[m], m);
        V *= dims[m];
        if (V > (1L << 28)) return fail(WL_ERR_DIMS, "volume exceeds 2^28 sites");
    }
    for (int k = 0; k < 8; ++k)
        if (!std::isfinite(phases[k])) return fail(WL_ERR_ARG, "non-finite boundary phase");
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev < 1) {
        (void)hipGetLastError();
        return fail(WL_ERR_HIP, "no HIP device available (%s)", hipGetErrorString(e));
    }
    int device = 0;
    HIP_TRY(hipGetDevice(&device));
    wl_ctx *c = new wl_ctx();
    std::memcpy(c->dims, dims, sizeof c->dims);
    std::memcpy(c->phases, phases, sizeof c->phases);
    c->V = V;
    c->Vh = V / 2;
    c->device = device;
    Geom &g = c->g;
    for (int m = 0; m < 4; ++m) g.L[m] = dims[m];
    g.lxh = dims[0] / 2;
    g.vh = (int)c->Vh;
    g.sy = g.lxh;
    g.sz = g.lxh * dims[1];
    g.st = g.lxh * dims[1] * dims[2];
    g.phase_mask = 0;
    for (int m = 0; m < 4; ++m) {
        g.zr[m] = phases[2 * m];
        g.zi[m] = phases[2 * m + 1];
        if (!(phases[2 * m] == 1.0 && phases[2 * m + 1] == 0.0)) g.phase_mask |= 1 << m;
    }
    // host packing of the canonical FP64 gauge field into the FP64 18-real internal layout
    const size_t slab = LinkIO<WL_F64, 18>::bytes_per_link * (size_t)padded(c->Vh);
    std::vector<double> host(slab / sizeof(double) * 8);
    for (long lex = 0; lex < V; ++lex) {
        long r = lex;
        const int x = (int)(r % dims[0]);
        r /= dims[0];
        const int y = (int)(r % dims[1]);
        r /= dims[1];
        const int z = (int)(r % dims[2]);
        const int t = (int)(r / dims[2]);
        const int par = (x + y + z + t) & 1;
        const long i = lex >> 1;
        for (int mu = 0; mu < 4; ++mu)
            for (int k = 0; k < 9; ++k) {
                const double *src = gauge_host + ((lex * 4 + mu) * 9 + k) * 2;
                // slab (par, mu); block i / 64, unit k, lane i % 64 (double2 units)
                double *dst = host.data() + (size_t)(par * 4 + mu) * (slab / sizeof(double)) +
                              ((size_t)((i >> 6) * 9 + k) * 64 + (i & 63)) * 2;
                dst[0] = src[0];
                dst[1] = src[1];
            }
    }
    void *d = nullptr;
    e = hipMalloc(&d, slab * 8);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        delete c;
        return fail(WL_ERR_NOMEM, "hipMalloc of gauge field failed: %s", hipGetErrorString(e));
    }
    e = hipMemcpy(d, host.data(), slab * 8, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(d);
        delete c;
        return fail(WL_ERR_HIP, "gauge upload failed: %s", hipGetErrorString(e));
    }
    c->gauge[WL_F64][0] = d;
    // measured defaults (MI355X, 24^3x48 and 32^3x64 lattices)
    c->cfg[WL_F64] = {128, 1, 2, WL_TCHUNK_AUTO, -1};
    c->cfg[WL_F32] = {128, 1, 2, WL_TCHUNK_AUTO, -1};
    c->cfg[WL_F16N] = {256, 1, 1, WL_TCHUNK_AUTO, -1};
    c->cfg[WL_BF16N] = {256, 1, 1, WL_TCHUNK_AUTO, -1};
    c->cfg[WL_I16N] = {256, 1, 1, WL_TCHUNK_AUTO, -1};
    c->slab[WL_F64][0] = slab;
    *out = c;
    return WL_OK;
}

extern "C" wl_status wl_ctx_destroy(wl_ctx *c) {
    if (!c) return WL_OK;
    (void)hipDeviceSynchronize();
    for (hipEvent_t e : c->event_pool) (void)hipEventDestroy(e);
    if (c->cg_exec) (void)hipGraphExecDestroy(c->cg_exec);
    if (c->cg_graph) (void)hipGraphDestroy(c->cg_graph);
    for (hipEvent_t e : c->handoff)
        if (e) (void)hipEventDestroy(e);
    if (c->own_stream) (void)hipStreamDestroy(c->own_stream);
    for (hipEvent_t e : c->halo_ev)
        if (e) (void)hipEventDestroy(e);
    if (c->comm_stream) (void)hipStreamDestroy(c->comm_stream);
    for (int p = 0; p < 5; ++p)
        for (int r = 0; r < 2; ++r)
            if (c->gauge[p][r]) (void)hipFree(c->gauge[p][r]);
    for (int s = 0; s < S_NSLOTS; ++s)
        if (c->buf[s]) (void)hipFree(c->buf[s]);
    if (c->host_pinned) (void)hipHostFree(c->host_pinned);
    delete c;
    return WL_OK;
}

static wl_status get_links(wl_ctx *c, int prec, int recon, const void **ptr, size_t *slab) {
    if (!recon_ok(prec, recon)) return fail(WL_ERR_UNSUPPORTED, "link format prec %d / recon %d not supported", prec, recon);
    const int ri = recon == 12 ? 1 : 0;
    if (!c->gauge[prec][ri]) {
        const size_t sl = link_bytes(prec, recon) * (size_t)padded(c->Vh);
        void *d = nullptr;
        hipError_t e = hipMalloc(&d, sl * 8);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(WL_ERR_NOMEM, "hipMalloc of link copy failed: %s", hipGetErrorString(e));
        }
        dim3 grid((unsigned)((c->Vh + 255) / 256), 8);
        const void *src = c->gauge[WL_F64][0];
        const size_t ss = c->slab[WL_F64][0];
        const int vh = (int)c->Vh;
        if (prec == WL_F64 && recon == 12) hipLaunchKernelGGL((k_link_convert<WL_F64, 12>), grid, dim3(256), 0, 0, d, sl, src, ss, vh);
        else if (prec == WL_F32 && recon == 18) hipLaunchKernelGGL((k_link_convert<WL_F32, 18>), grid, dim3(256), 0, 0, d, sl, src, ss, vh);
        else if (prec == WL_F32 && recon == 12) hipLaunchKernelGGL((k_link_convert<WL_F32, 12>), grid, dim3(256), 0, 0, d, sl, src, ss, vh);
        else if (prec == WL_F16N) hipLaunchKernelGGL((k_link_convert<WL_F16N, 12>), grid, dim3(256), 0, 0, d, sl, src, ss, vh);
        else if (prec == WL_BF16N) hipLaunchKernelGGL((k_link_convert<WL_BF16N, 12>), grid, dim3(256), 0, 0, d, sl, src, ss, vh);
        else if (prec == WL_I16N) hipLaunchKernelGGL((k_link_convert<WL_I16N, 12>), grid, dim3(256), 0, 0, d, sl, src, ss, vh);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipDeviceSynchronize());
        c->gauge[prec][ri] = d;
        c->slab[prec][ri] = sl;
    }
    *ptr = c->gauge[prec][ri];
    *slab = c->slab[prec][ri];
    return WL_OK;
}

extern "C" wl_status wl_ctx_prepare_links(wl_ctx *c, wl_prec prec, int recon) {
    g_err.clear();
    if (!c) return fail(WL_ERR_ARG, "null context");
    if (!prec_ok(prec)) return fail(WL_ERR_ARG, "bad precision %d", (int)prec);
    const void *p;
    size_t s;
    return get_links(c, prec, recon, &p, &s);
}

extern "C" wl_status wl_spinor_bytes(const wl_ctx *c, wl_subset subset, wl_prec prec, int nrhs, size_t *bytes) {
    g_err.clear();
    wl_status st = check_field_args(c, subset, prec, nrhs);
    if (st) return st;
    if (!bytes) return fail(WL_ERR_ARG, "null output");
    *bytes = half_bytes(c, prec, nrhs) * (subset == WL_FULL ? 2 : 1);
    return WL_OK;
}

extern "C" wl_status wl_pack_spinor(const wl_ctx *c, void *dst, const double *src, wl_subset subset, wl_prec prec,
                                    int nrhs, void *stream) {
    g_err.clear();
    wl_status st = check_field_args(c, subset, prec, nrhs);
    if (st) return st;
    if (!dst || !src) return fail(WL_ERR_ARG, "null field pointer");
    if (!aligned16(dst) || !aligned16(src)) return fail(WL_ERR_ARG, "field pointers must be 16-byte aligned");
    const int nh = subset == WL_FULL ? 2 : 1;
    const size_t hb = half_bytes(c, prec, nrhs);
    if (overlap(dst, hb * nh, src, (size_t)c->Vh * nh * nrhs * 24 * 8)) return fail(WL_ERR_ARG, "dst and src overlap");
    dim3 grid((unsigned)((c->Vh * nrhs + 255) / 256), nh);
    HIP_TRY((launch_prec<PackK>(prec, grid, (hipStream_t)stream, c->g, dst, hb, src, (int)subset, nrhs)));
    return WL_OK;
}

extern "C" wl_status wl_unpack_spinor(const wl_ctx *c, double *dst, const void *src, wl_subset subset, wl_prec prec,
                                      int nrhs, void *stream) {
    g_err.clear();
    wl_status st = check_field_args(c, subset, prec, nrhs);
    if (st) return st;
    if (!dst || !src) return fail(WL_ERR_ARG, "null field pointer");
    if (!aligned16(dst) || !aligned16(src)) return fail(WL_ERR_ARG, "field pointers must be 16-byte aligned");
    const int nh = subset == WL_FULL ? 2 : 1;
    const size_t hb = half_bytes(c, prec, nrhs);
    if (overlap(dst, (size_t)c->Vh * nh * nrhs * 24 * 8, src, hb * nh)) return fail(WL_ERR_ARG, "dst and src overlap");
    dim3 grid((unsigned)((c->Vh * nrhs + 255) / 256), nh);
    HIP_TRY((launch_prec<UnpackK>(prec, grid, (hipStream_t)stream, c->g, dst, src, hb, (int)subset, nrhs)));
    return WL_OK;
}

static VecArgs vec_args(const wl_ctx *c, int prec, int nrhs) {
    VecArgs a;
    std::memset(&a, 0, sizeof a);
    a.n = c->Vh * (long)nrhs;
    a.nrhs = nrhs;
    (void)prec;
    return a;
}
static void set_vec(VecArgs &a, int k, const void *base, size_t hb) {
    a.v[k][0] = (void *)base;
    a.v[k][1] = (char *)base + hb;
}

extern "C" wl_status wl_convert_spinor(const wl_ctx *c, void *dst, wl_prec dprec, const void *src, wl_prec sprec,
                                       wl_subset subset, int nrhs, void *stream) {
    g_err.clear();
    wl_status st = check_field_args(c, subset, sprec, nrhs);
    if (st) return st;
    if (!prec_ok(dprec)) return fail(WL_ERR_ARG, "bad precision %d", (int)dprec);
    if (!dst || !src || !aligned16(dst) || !aligned16(src)) return fail(WL_ERR_ARG, "null or misaligned field pointer");
    const int nh = subset == WL_FULL ? 2 : 1;
    if (overlap(dst, half_bytes(c, dprec, nrhs) * nh, src, half_bytes(c, sprec, nrhs) * nh))
        return fail(WL_ERR_ARG, "dst and src overlap");
    VecArgs a = vec_args(c, sprec, nrhs);
    set_vec(a, 0, src, half_bytes(c, sprec, nrhs));
    set_vec(a, 1, dst, half_bytes(c, dprec, nrhs));
    HIP_TRY(blas_convert(dprec, sprec, false, a, nh, (hipStream_t)stream));
    return WL_OK;
}

// ------------------------------------------------------------------ operators
// Enqueue out = a x + b H in (or H^+) for one output subset.
// HopArgs of out = a x + b H in for one output subset; *np = output parities
static wl_status fill_hop_args(wl_ctx *c, int prec, int recon, void *out, const void *in, const void *x,
                               int out_subset, int nrhs, double a, double b, double *partials, long part_stride,
                               const int *flag, HopArgs &h, int *np_out, double tm_x = 0.0, double tm_h = 0.0) {
    const void *gauge;
    size_t slab;
    wl_status st = get_links(c, prec, recon, &gauge, &slab);
    if (st) return st;
    const size_t hb = half_bytes(c, prec, nrhs);
    std::memset(&h, 0, sizeof h);
    h.g = c->g;
    h.gauge = gauge;
    h.slab_bytes = slab;
    h.nrhs = nrhs;
    h.npts = c->Vh * (long)nrhs;
    h.a = a;
    h.b = b;
    h.tm_x = tm_x;
    h.tm_h = tm_h;
    h.partials = partials;
    h.part_stride = part_stride;
    h.flag = flag;
    int np = 1;
    if (out_subset == WL_FULL) {
        h.out[0] = out;
        h.out[1] = (char *)out + hb;
        h.in[0] = in;
        h.in[1] = (const char *)in + hb;
        if (x) {
            h.x[0] = x;
            h.x[1] = (const char *)x + hb;
        }
        h.out_par0 = 0;
        np = 2;
    } else {
        const int p = out_subset;
        h.out[p] = out;
        h.in[1 - p] = in;
        h.x[p] = x;
        h.out_par0 = p;
    }
    *np_out = np;
    return WL_OK;
}

// EPI_CGR: the residual r (the output's subset and storage) updated in place with
// alpha of rhs k read from sc[k]
static void set_cg_residual(const wl_ctx *c, int prec, int nrhs, int out_subset, void *cg_r, const CGScalars *cg_sc,
                            HopArgs &h) {
    const size_t hb = half_bytes(c, prec, nrhs);
    if (out_subset == WL_FULL) {
        h.r[0] = cg_r;
        h.r[1] = (char *)cg_r + hb;
    } else {
        h.r[out_subset] = cg_r;
    }
    h.alpha = (const char *)cg_sc + offsetof(CGScalars, alpha);
    h.alpha_stride = sizeof(CGScalars);
}

static wl_status hop_core(wl_ctx *c, int prec, int recon, bool dag, int epi, void *out, const void *in,
                          const void *x, int out_subset, int nrhs, double a, double b, double *partials,
                          long part_stride, const int *flag, hipStream_t s, long *nblk_out = nullptr,
                          double tm_x = 0.0, double tm_h = 0.0, void *cg_r = nullptr,
                          const CGScalars *cg_sc = nullptr) {
    HopArgs h;
    int np = 1;
    wl_status st = fill_hop_args(c, prec, recon, out, in, x, out_subset, nrhs, a, b, partials, part_stride, flag, h,
                                 &np, tm_x, tm_h);
    if (st) return st;
    if (epi & EPI_CGR) set_cg_residual(c, prec, nrhs, out_subset, cg_r, cg_sc, h);
    hipEvent_t *ev = nullptr;
    if (c->timing && !c->capturing && c->timed.size() < (1u << 16) && c->timing_seq++ % c->timing_stride == 0) {
        if (c->pool_used + 2 > c->event_pool.size()) {
            for (int k = 0; k < 256; ++k) {
                hipEvent_t e;
                HIP_TRY(hipEventCreate(&e));
                c->event_pool.push_back(e);
            }
        }
        c->timed.push_back({timing_key(prec, recon, dag, epi),
                            {c->event_pool[c->pool_used], c->event_pool[c->pool_used + 1]},
                            c->timing_iter, c->timing_cycle});
        c->pool_used += 2;
        ev = c->timed.back().ev;
        HIP_TRY(hipEventRecord(ev[0], s));
    }
    const LaunchCfg &cfg = c->cfg[prec];
    HIP_TRY(launch_hop(prec, recon, dag, epi, h, np, cfg, s));
    if (ev) HIP_TRY(hipEventRecord(ev[1], s));
    if (nblk_out) *nblk_out = hop_launch_blocks(effective_tps(prec, cfg), cfg, h.npts, nrhs) * np;
    return WL_OK;
}

static wl_status dslash_common(const wl_ctx *cc, void *out, const void *in, wl_subset subset, wl_prec prec, int recon,
                               int nrhs, void *stream, bool dag) {
    g_err.clear();
    wl_ctx *c = const_cast<wl_ctx *>(cc);
    wl_status st = check_field_args(c, subset, prec, nrhs);
    if (st) return st;
    if (!recon_ok(prec, recon)) return fail(WL_ERR_UNSUPPORTED, "prec %d with recon %d not supported", prec, recon);
    if (!out || !in || !aligned16(out) || !aligned16(in)) return fail(WL_ERR_ARG, "null or misaligned field pointer");
    const size_t bytes = half_bytes(c, prec, nrhs) * (subset == WL_FULL ? 2 : 1);
    if (overlap(out, bytes, in, bytes)) return fail(WL_ERR_ARG, "out and in overlap");
    return hop_core(c, prec, recon, dag, 0, out, in, nullptr, subset, nrhs, 0.0, 1.0, nullptr, 0, nullptr,
                    (hipStream_t)stream);
}

extern "C" wl_status wl_dslash_apply(const wl_ctx *c, void *out, const void *in, wl_subset subset, wl_prec prec,
                                     int recon, int nrhs, void *stream) {
    return dslash_common(c, out, in, subset, prec, recon, nrhs, stream, false);
}
// Bulk / boundary split of the hopping term with the t-faces exchanged through
// buffers on a second stream while the bulk is computed (the paper's overlap
// scheme; on one device the faces of the periodic lattice go to itself).
extern "C" wl_status wl_dslash_apply_split(const wl_ctx *cc, void *out, const void *in, wl_subset subset,
                                           wl_prec prec, int recon, int dagger, void *stream) {
    g_err.clear();
    wl_ctx *c = const_cast<wl_ctx *>(cc);
    if (subset != WL_EVEN && subset != WL_ODD) return fail(WL_ERR_ARG, "the split form takes one output parity");
    wl_status st = check_field_args(c, subset, prec, 1);
    if (st) return st;
    if (prec != WL_F64 && prec != WL_F32) return fail(WL_ERR_UNSUPPORTED, "the split form needs FP64 or FP32 storage");
    if (!recon_ok(prec, recon)) return fail(WL_ERR_UNSUPPORTED, "prec %d with recon %d not supported", prec, recon);
    if (!out || !in || !aligned16(out) || !aligned16(in)) return fail(WL_ERR_ARG, "null or misaligned field pointer");
    const size_t hb = half_bytes(c, prec, 1);
    if (overlap(out, hb, in, hb)) return fail(WL_ERR_ARG, "out and in overlap");
    HopArgs h;
    int np = 1;
    if ((st = fill_hop_args(c, prec, recon, out, in, nullptr, subset, 1, 0.0, 1.0, nullptr, 0, nullptr, h, &np)))
        return st;
    const size_t fb = (size_t)6 * c->g.st * (prec == WL_F64 ? 16 : 8);  // one face buffer
    const size_t fba = (fb + 255) & ~(size_t)255;
    if ((st = ensure_buf(c, S_FACE, 4 * fba))) return st;
    char *fbase = (char *)c->buf[S_FACE];
    void *send_fwd = fbase, *send_bwd = fbase + fba, *recv_fwd = fbase + 2 * fba, *recv_bwd = fbase + 3 * fba;
    if (!c->comm_stream) {
        HIP_TRY(hipStreamCreateWithFlags(&c->comm_stream, hipStreamNonBlocking));
        HIP_TRY(hipEventCreateWithFlags(&c->halo_ev[0], hipEventDisableTiming));
        HIP_TRY(hipEventCreateWithFlags(&c->halo_ev[1], hipEventDisableTiming));
    }
    hipStream_t s = (hipStream_t)stream;
    const bool dag = dagger != 0;
    const int par = subset;
    // faces first; their transfer runs on the comm stream while the bulk computes
    HIP_TRY(launch_face_pack(prec, recon, dag, h, par, send_fwd, send_bwd, s));
    HIP_TRY(hipEventRecord(c->halo_ev[0], s));
    HIP_TRY(hipStreamWaitEvent(c->comm_stream, c->halo_ev[0], 0));
    HIP_TRY(hipMemcpyAsync(recv_fwd, send_fwd, fb, hipMemcpyDeviceToDevice, c->comm_stream));
    HIP_TRY(hipMemcpyAsync(recv_bwd, send_bwd, fb, hipMemcpyDeviceToDevice, c->comm_stream));
    HIP_TRY(hipEventRecord(c->halo_ev[1], c->comm_stream));
    h.swizzle = c->cfg[prec].swizzle;
    set_processing_order(h, c->cfg[prec].tchunk);
    HIP_TRY(launch_hop_bulk(prec, recon, dag, use_nontemporal(prec, c->cfg[prec], h, 1, 0), h, par, s));
    HIP_TRY(hipStreamWaitEvent(s, c->halo_ev[1], 0));
    HIP_TRY(launch_hop_boundary(prec, recon, dag, h, par, recv_fwd, recv_bwd, s));
    return WL_OK;
}

extern "C" wl_status wl_dslash_dagger_apply(const wl_ctx *c, void *out, const void *in, wl_subset subset,
                                            wl_prec prec, int recon, int nrhs, void *stream) {
    return dslash_common(c, out, in, subset, prec, recon, nrhs, stream, true);
}

// out = M in (M^+ if dag); tmp: odd half temporary for DHAT.  Norm partials of
// out if partials != null.  With a twisted mass mu the site-diagonal part is
// A = 1 + i nu gamma_5, nu = 2 kappa mu (A^+ for M^+): D = A - kappa H and
// D_hat = A - kappa^2 H_eo A^-1 H_oe, A^-1 = (1 - i nu gamma_5) / (1 + nu^2).
static wl_status apply_m(wl_ctx *c, int op, bool dag, double kappa, int prec, int recon, int nrhs, void *out,
                         const void *in, void *tmp, double *partials, long stride, const int *flag, hipStream_t s,
                         long *nblk, double mu = 0.0) {
    const int epi = EPI_XPAY | (partials ? EPI_NORM : 0);
    const double nu = (dag ? -2.0 : 2.0) * kappa * mu;
    if (op == WL_OP_D)
        return hop_core(c, prec, recon, dag, epi, out, in, in, WL_FULL, nrhs, 1.0, -kappa, partials, stride, flag, s,
                        nblk, nu, 0.0);
    wl_status st = hop_core(c, prec, recon, dag, 0, tmp, in, nullptr, WL_ODD, nrhs, 0.0, 1.0 / (1.0 + nu * nu),
                            nullptr, 0, flag, s, nullptr, 0.0, -nu);
    if (st) return st;
    return hop_core(c, prec, recon, dag, epi, out, tmp, in, WL_EVEN, nrhs, 1.0, -kappa * kappa, partials, stride,
                    flag, s, nblk, nu, 0.0);
}

// r -= alpha M^+ in with ||r||^2 partials (the last stage of CG's A p, fused with the
// residual update; alpha per rhs from sc): the operator applications of apply_m(dag)
// with the final one's result folded into r instead of being stored.
static wl_status apply_mdag_update_r(wl_ctx *c, int op, double kappa, int prec, int recon, int nrhs, void *r,
                                     const void *in, void *tmp, double *partials, long stride, const int *flag,
                                     hipStream_t s, long *nblk, double mu, const CGScalars *sc) {
    const int epi = EPI_XPAY | EPI_NORM | EPI_CGR;
    const double nu = -2.0 * kappa * mu;
    if (op == WL_OP_D)
        return hop_core(c, prec, recon, true, epi, r, in, in, WL_FULL, nrhs, 1.0, -kappa, partials, stride, flag, s,
                        nblk, nu, 0.0, r, sc);
    wl_status st = hop_core(c, prec, recon, true, 0, tmp, in, nullptr, WL_ODD, nrhs, 0.0, 1.0 / (1.0 + nu * nu),
                            nullptr, 0, flag, s, nullptr, 0.0, -nu);
    if (st) return st;
    return hop_core(c, prec, recon, true, epi, r, tmp, in, WL_EVEN, nrhs, 1.0, -kappa * kappa, partials, stride, flag,
                    s, nblk, nu, 0.0, r, sc);
}

static wl_status dirac_common(wl_ctx *c, void *out, const void *in, wl_op op, int dagger, double kappa, double mu,
                              wl_prec prec, int recon, int nrhs, void *stream) {
    g_err.clear();
    if (op != WL_OP_D && op != WL_OP_DHAT) return fail(WL_ERR_ARG, "bad operator %d", (int)op);
    const int subset = op == WL_OP_D ? WL_FULL : WL_EVEN;
    wl_status st = check_field_args(c, subset, prec, nrhs);
    if (st) return st;
    if (!recon_ok(prec, recon)) return fail(WL_ERR_UNSUPPORTED, "prec %d with recon %d not supported", prec, recon);
    if (!out || !in || !aligned16(out) || !aligned16(in)) return fail(WL_ERR_ARG, "null or misaligned field pointer");
    if (!std::isfinite(kappa) || !std::isfinite(mu)) return fail(WL_ERR_ARG, "non-finite kappa or mu");
    const size_t hb = half_bytes(c, prec, nrhs);
    const size_t bytes = hb * (op == WL_OP_D ? 2 : 1);
    if (overlap(out, bytes, in, bytes)) return fail(WL_ERR_ARG, "out and in overlap");
    void *tmp = nullptr;
    if (op == WL_OP_DHAT) {
        st = ensure_buf(c, S_TMP_OP, hb);
        if (st) return st;
        tmp = c->buf[S_TMP_OP];
    }
    return apply_m(c, op, dagger != 0, kappa, prec, recon, nrhs, out, in, tmp, nullptr, 0, nullptr,
                   (hipStream_t)stream, nullptr, mu);
}

extern "C" wl_status wl_dirac_apply(wl_ctx *c, void *out, const void *in, wl_op op, int dagger, double kappa,
                                    wl_prec prec, int recon, int nrhs, void *stream) {
    return dirac_common(c, out, in, op, dagger, kappa, 0.0, prec, recon, nrhs, stream);
}

extern "C" wl_status wl_dirac_tm_apply(wl_ctx *c, void *out, const void *in, wl_op op, int dagger, double kappa,
                                       double mu, wl_prec prec, int recon, int nrhs, void *stream) {
    return dirac_common(c, out, in, op, dagger, kappa, mu, prec, recon, nrhs, stream);
}

static wl_status eo_helper(const wl_ctx *cc, void *out, const void *a_in, const void *hop_in, int out_subset,
                           double kappa, wl_prec prec, int recon, int nrhs, void *stream) {
    g_err.clear();
    wl_ctx *c = const_cast<wl_ctx *>(cc);
    wl_status st = check_field_args(c, out_subset, prec, nrhs);
    if (st) return st;
    if (!recon_ok(prec, recon)) return fail(WL_ERR_UNSUPPORTED, "prec %d with recon %d not supported", prec, recon);
    if (!out || !a_in || !hop_in || !aligned16(out) || !aligned16(a_in) || !aligned16(hop_in))
        return fail(WL_ERR_ARG, "null or misaligned field pointer");
    if (!std::isfinite(kappa)) return fail(WL_ERR_ARG, "non-finite kappa");
    const size_t hb = half_bytes(c, prec, nrhs);
    if (overlap(out, hb, hop_in, hb)) return fail(WL_ERR_ARG, "output overlaps the hopping input");
    return hop_core(c, prec, recon, false, EPI_XPAY, out, hop_in, a_in, out_subset, nrhs, 1.0, kappa, nullptr, 0,
                    nullptr, (hipStream_t)stream);
}

extern "C" wl_status wl_eo_prepare(const wl_ctx *c, void *bhat_e, const void *b_e, const void *b_o, double kappa,
                                   wl_prec prec, int recon, int nrhs, void *stream) {
    return eo_helper(c, bhat_e, b_e, b_o, WL_EVEN, kappa, prec, recon, nrhs, stream);
}
extern "C" wl_status wl_eo_reconstruct(const wl_ctx *c, void *x_o, const void *x_e, const void *b_o, double kappa,
                                       wl_prec prec, int recon, int nrhs, void *stream) {
    return eo_helper(c, x_o, b_o, x_e, WL_ODD, kappa, prec, recon, nrhs, stream);
}

// twisted mass: bhat_e = b_e + kappa H_eo A^-1 b_o ; x_o = A^-1 (b_o + kappa H_oe x_e)
extern "C" wl_status wl_eo_prepare_tm(const wl_ctx *cc, void *bhat_e, const void *b_e, const void *b_o, double kappa,
                                      double mu, wl_prec prec, int recon, int nrhs, void *stream) {
    g_err.clear();
    wl_ctx *c = const_cast<wl_ctx *>(cc);
    wl_status st = check_field_args(c, WL_ODD, prec, nrhs);
    if (st) return st;
    if (!b_o || !aligned16(b_o)) return fail(WL_ERR_ARG, "null or misaligned field pointer");
    if (!std::isfinite(kappa) || !std::isfinite(mu)) return fail(WL_ERR_ARG, "non-finite kappa or mu");
    const size_t hb = half_bytes(c, prec, nrhs);
    if ((st = ensure_buf(c, S_TMP_OP, hb))) return st;
    const double nu = 2.0 * kappa * mu;
    VecArgs v = vec_args(c, prec, nrhs);
    set_vec(v, 0, b_o, hb);
    set_vec(v, 1, c->buf[S_TMP_OP], hb);
    v.a = 1.0 / (1.0 + nu * nu);
    v.b = -nu;
    HIP_TRY(blas_twist(prec, v, 1, (hipStream_t)stream));
    return eo_helper(c, bhat_e, b_e, c->buf[S_TMP_OP], WL_EVEN, kappa, prec, recon, nrhs, stream);
}

extern "C" wl_status wl_eo_reconstruct_tm(const wl_ctx *cc, void *x_o, const void *x_e, const void *b_o,
                                          double kappa, double mu, wl_prec prec, int recon, int nrhs, void *stream) {
    g_err.clear();
    wl_ctx *c = const_cast<wl_ctx *>(cc);
    wl_status st = check_field_args(c, WL_ODD, prec, nrhs);
    if (st) return st;
    if (!recon_ok(prec, recon)) return fail(WL_ERR_UNSUPPORTED, "prec %d with recon %d not supported", prec, recon);
    if (!x_o || !x_e || !b_o || !aligned16(x_o) || !aligned16(x_e) || !aligned16(b_o))
        return fail(WL_ERR_ARG, "null or misaligned field pointer");
    if (!std::isfinite(kappa) || !std::isfinite(mu)) return fail(WL_ERR_ARG, "non-finite kappa or mu");
    const size_t hb = half_bytes(c, prec, nrhs);
    if (overlap(x_o, hb, x_e, hb)) return fail(WL_ERR_ARG, "output overlaps the hopping input");
    const double nu = 2.0 * kappa * mu, sc = 1.0 / (1.0 + nu * nu);
    // (1 - i nu gamma_5) / (1 + nu^2) applied to both terms of the epilogue
    return hop_core(c, prec, recon, false, EPI_XPAY, x_o, x_e, b_o, WL_ODD, nrhs, sc, kappa * sc, nullptr, 0, nullptr,
                    (hipStream_t)stream, nullptr, -nu, -nu);
}

// ------------------------------------------------------------------ BLAS API
static long part_stride_for(const wl_ctx *c, int nrhs) {
    const long n = c->Vh * (long)nrhs;
    const long hb = hop_blocks(n, 64, 2) * 2;  // the most blocks any hopping launch may use
    const long bb = blas_blocks(n) * 2;
    return std::max(hb, bb);
}

extern "C" wl_status wl_blas_axpy(const wl_ctx *c, double a, const void *x, void *y, wl_subset subset, wl_prec prec,
                                  int nrhs, void *stream) {
    g_err.clear();
    wl_status st = check_field_args(c, subset, prec, nrhs);
    if (st) return st;
    if (!x || !y || !aligned16(x) || !aligned16(y)) return fail(WL_ERR_ARG, "null or misaligned field pointer");
    if (!std::isfinite(a)) return fail(WL_ERR_ARG, "non-finite scalar");
    VecArgs v = vec_args(c, prec, nrhs);
    const size_t hb = half_bytes(c, prec, nrhs);
    set_vec(v, 0, x, hb);
    set_vec(v, 1, y, hb);
    v.a = a;
    v.b = 1.0;
    HIP_TRY(blas_axpby(prec, v, subset == WL_FULL ? 2 : 1, false, (hipStream_t)stream));
    return WL_OK;
}

static wl_status reduce_to_host(wl_ctx *c, int nvals, long stride, long nblk, double *out, hipStream_t s) {
    wl_status st = ensure_buf(c, S_SCAL, std::max<size_t>(c->buf_bytes[S_SCAL], 64 * sizeof(double) * 2));
    if (st) return st;
    double *d = (double *)c->buf[S_SCAL];
    HIP_TRY(reduce_partials((const double *)c->buf[S_PARTIALS], stride, nblk, nvals, d, s));
    HIP_TRY(hipMemcpyAsync(out, d, nvals * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return WL_OK;
}

extern "C" wl_status wl_blas_dot(const wl_ctx *cc, const void *x, const void *y, wl_subset subset, wl_prec prec,
                                 int nrhs, double result[2], void *stream) {
    g_err.clear();
    wl_ctx *c = const_cast<wl_ctx *>(cc);
    wl_status st = check_field_args(c, subset, prec, nrhs);
    if (st) return st;
    if (!x || !y || !result || !aligned16(x) || !aligned16(y)) return fail(WL_ERR_ARG, "null or misaligned pointer");
    const long stride = part_stride_for(c, nrhs);
    st = ensure_buf(c, S_PARTIALS, sizeof(double) * 2 * nrhs * stride);
    if (st) return st;
    VecArgs v = vec_args(c, prec, nrhs);
    const size_t hb = half_bytes(c, prec, nrhs);
    set_vec(v, 0, x, hb);
    set_vec(v, 1, y, hb);
    v.partials = (double *)c->buf[S_PARTIALS];
    v.part_stride = stride;
    const int nh = subset == WL_FULL ? 2 : 1;
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(blas_dot(prec, v, nh, s));
    std::vector<double> vals(2 * nrhs);
    st = reduce_to_host(c, 2 * nrhs, stride, blas_blocks(v.n) * nh, vals.data(), s);
    if (st) return st;
    // result holds (re, im) for rhs 0; callers with nrhs > 1 get the sum over rhs
    double re = 0, im = 0;
    for (int r = 0; r < nrhs; ++r) {
        re += vals[r];
        im += vals[nrhs + r];
    }
    result[0] = re;
    result[1] = im;
    return WL_OK;
}

extern "C" wl_status wl_blas_norm2(const wl_ctx *cc, const void *x, wl_subset subset, wl_prec prec, int nrhs,
                                   double *result, void *stream) {
    g_err.clear();
    wl_ctx *c = const_cast<wl_ctx *>(cc);
    wl_status st = check_field_args(c, subset, prec, nrhs);
    if (st) return st;
    if (!x || !result || !aligned16(x)) return fail(WL_ERR_ARG, "null or misaligned pointer");
    const long stride = part_stride_for(c, nrhs);
    st = ensure_buf(c, S_PARTIALS, sizeof(double) * 2 * nrhs * stride);
    if (st) return st;
    VecArgs v = vec_args(c, prec, nrhs);
    set_vec(v, 0, x, half_bytes(c, prec, nrhs));
    v.partials = (double *)c->buf[S_PARTIALS];
    v.part_stride = stride;
    const int nh = subset == WL_FULL ? 2 : 1;
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(blas_norm2(prec, v, nh, s));
    std::vector<double> vals(nrhs);
    st = reduce_to_host(c, nrhs, stride, blas_blocks(v.n) * nh, vals.data(), s);
    if (st) return st;
    double t = 0;
    for (double q : vals) t += q;
    *result = t;
    return WL_OK;
}

// ------------------------------------------------------------------ CG
extern "C" void wl_solver_params_default(wl_solver_params *p) {
    if (!p) return;
    p->tol = 1e-10;
    p->maxiter = 100000;
    p->check_every = 25;
    p->max_restarts = 5;
    p->prec = WL_F64;
    p->recon = 18;
    p->reliable_every = 100;
    p->reliable_delta = 0.1;
    p->use_graph = 0;
    p->ru_restart = -1;
    p->mu = 0.0;
}

namespace {
struct CGRun {
    wl_ctx *c;
    int op, nrhs, prec, recon, nh;
    double kappa;
    hipStream_t s;
    size_t hb_lo, hb_hi;
    void *x, *r, *p, *q, *sv, *tmp;  // inner precision (x is FP64)
    // mixed precision: the fused iterations add alpha p to this FP32 field, which
    // true_residual folds into x (the only reader of x) before it uses x
    void *xlo;
    size_t hb_xlo;
    const void *b;
    void *rhi, *thi, *tmphi;
    double *partials;
    long stride;
    CGScalars *sc;
    double *bnorm2;
    int *done;
    long nblk_blas;
    int ru_restart;
    double mu;  // twisted mass (0: Wilson)
};
}  // namespace

// x += x_lo, x_lo = 0 (mixed precision; every read of x follows this)
static wl_status fold_x(CGRun &R) {
    if (!R.xlo) return WL_OK;
    VecArgs v = vec_args(R.c, WL_F32, R.nrhs);
    set_vec(v, 0, R.xlo, R.hb_xlo);
    set_vec(v, 1, R.x, R.hb_hi);
    HIP_TRY(blas_convert(WL_F64, WL_F32, true, v, R.nh, R.s));
    VecArgs z = vec_args(R.c, WL_F32, R.nrhs);
    set_vec(z, 0, R.xlo, R.hb_xlo);
    HIP_TRY(blas_zero(WL_F32, z, R.nh, R.s));
    return WL_OK;
}

// t = A x = M^+ M x in FP64; r_hi = b - t; partials of ||r_hi||^2
static wl_status true_residual(CGRun &R) {
    wl_status st = fold_x(R);
    if (st) return st;
    st = apply_m(R.c, R.op, false, R.kappa, WL_F64, 18, R.nrhs, R.thi, R.x, R.tmphi, nullptr, 0, nullptr,
                           R.s, nullptr, R.mu);
    if (st) return st;
    st = apply_m(R.c, R.op, true, R.kappa, WL_F64, 18, R.nrhs, R.rhi, R.thi, R.tmphi, nullptr, 0, nullptr, R.s,
                 nullptr, R.mu);
    if (st) return st;
    VecArgs v = vec_args(R.c, WL_F64, R.nrhs);
    set_vec(v, 0, R.b, R.hb_hi);
    set_vec(v, 1, R.rhi, R.hb_hi);
    set_vec(v, 2, R.rhi, R.hb_hi);
    v.partials = R.partials;
    v.part_stride = R.stride;
    HIP_TRY(blas_residual(WL_F64, v, R.nh, R.s));
    return WL_OK;
}

// r_lo = r_hi ; p = r_lo
static wl_status load_residual(CGRun &R) {
    VecArgs v = vec_args(R.c, R.prec, R.nrhs);
    if (R.prec != WL_F64) {
        set_vec(v, 0, R.rhi, R.hb_hi);
        set_vec(v, 1, R.r, R.hb_lo);
        HIP_TRY(blas_convert(R.prec, WL_F64, false, v, R.nh, R.s));
    }
    set_vec(v, 0, R.r, R.hb_lo);
    set_vec(v, 1, R.p, R.hb_lo);
    HIP_TRY(blas_convert(R.prec, R.prec, false, v, R.nh, R.s));
    return WL_OK;
}

// the part of a CG iteration after the operator applications (q = M p, whose
// norm gave alpha, and sv = M^+ q = A p): x += alpha p, r -= alpha sv, the
// optional FP64 refresh of r, beta, p = r + beta p
static wl_status cg_finish_iteration(CGRun &R, bool reliable) {
    VecArgs v = vec_args(R.c, R.prec, R.nrhs);
    set_vec(v, 0, R.x, R.hb_hi);
    set_vec(v, 1, R.p, R.hb_lo);
    set_vec(v, 2, R.r, R.hb_lo);
    set_vec(v, 3, R.sv, R.hb_lo);
    v.partials = R.partials;
    v.part_stride = R.stride;
    v.sc = R.sc;
    v.flag = R.done;
    HIP_TRY(cg_update_xr(R.prec, WL_F64, v, R.nh, R.s));
    if (reliable) {
        // replace the iterated residual by the FP64 one before the step length of p is
        // formed; its norm is kept first (the beta step compares the two)
        HIP_TRY(cg_stash_rho(R.sc, R.nrhs, R.partials, R.stride, R.nblk_blas, R.done, R.s));
        wl_status st = true_residual(R);
        if (st) return st;
        VecArgs w = vec_args(R.c, R.prec, R.nrhs);
        set_vec(w, 0, R.rhi, R.hb_hi);
        set_vec(w, 1, R.r, R.hb_lo);
        w.flag = R.done;
        HIP_TRY(blas_convert(R.prec, WL_F64, false, w, R.nh, R.s));
    }
    HIP_TRY(cg_beta(R.sc, R.nrhs, R.partials, R.stride, R.nblk_blas, R.done,
                    reliable ? (R.ru_restart ? 2 : 1) : 0, R.s));
    VecArgs u = vec_args(R.c, R.prec, R.nrhs);
    set_vec(u, 0, R.r, R.hb_lo);
    set_vec(u, 1, R.p, R.hb_lo);
    u.sc = R.sc;
    u.flag = R.done;
    HIP_TRY(cg_update_p(R.prec, u, R.nh, R.s));
    return WL_OK;
}

static wl_status cg_iteration(CGRun &R, bool reliable) {
    long nblk = 0;
    wl_status st = apply_m(R.c, R.op, false, R.kappa, R.prec, R.recon, R.nrhs, R.q, R.p, R.tmp, R.partials, R.stride,
                           R.done, R.s, &nblk, R.mu);
    if (st) return st;
    HIP_TRY(cg_alpha(R.sc, R.nrhs, R.partials, R.stride, nblk, R.done, R.s));
    const LaunchCfg &cfg = R.c->cfg[R.prec];
    if (!reliable && effective_rpt(cfg, R.nrhs, effective_tps(R.prec, cfg)) == 1) {
        // the last operator stage updates r in place (r -= alpha A p, ||r||^2) instead of
        // storing A p; then x += alpha p and p = r + beta p in one pass
        long nblk2 = 0;
        if ((st = apply_mdag_update_r(R.c, R.op, R.kappa, R.prec, R.recon, R.nrhs, R.r, R.q, R.tmp, R.partials,
                                      R.stride, R.done, R.s, &nblk2, R.mu, R.sc)))
            return st;
        HIP_TRY(cg_beta(R.sc, R.nrhs, R.partials, R.stride, nblk2, R.done, 0, R.s));
        VecArgs u = vec_args(R.c, R.prec, R.nrhs);
        set_vec(u, 0, R.xlo ? R.xlo : R.x, R.xlo ? R.hb_xlo : R.hb_hi);
        set_vec(u, 1, R.p, R.hb_lo);
        set_vec(u, 2, R.r, R.hb_lo);
        u.sc = R.sc;
        u.flag = nullptr;  // must also run after the last system's final step
        HIP_TRY(cg_update_xp(R.prec, R.xlo ? WL_F32 : WL_F64, u, R.nh, R.s));
        return WL_OK;
    }
    st = apply_m(R.c, R.op, true, R.kappa, R.prec, R.recon, R.nrhs, R.sv, R.q, R.tmp, nullptr, 0, R.done, R.s,
                 nullptr, R.mu);
    if (st) return st;
    return cg_finish_iteration(R, reliable);
}

// Everything one plain iteration depends on; a captured graph is reused only
// while this key is unchanged.
static std::vector<uintptr_t> graph_key(const CGRun &R) {
    const LaunchCfg &g = R.c->cfg[R.prec];
    uint64_t kb, mb;
    std::memcpy(&kb, &R.kappa, sizeof kb);
    std::memcpy(&mb, &R.mu, sizeof mb);
    return {(uintptr_t)R.op, (uintptr_t)R.prec, (uintptr_t)R.recon, (uintptr_t)R.nrhs, (uintptr_t)kb, (uintptr_t)mb,
            (uintptr_t)R.x, (uintptr_t)R.xlo, (uintptr_t)R.r, (uintptr_t)R.p, (uintptr_t)R.q, (uintptr_t)R.sv,
            (uintptr_t)R.tmp,
            (uintptr_t)R.partials, (uintptr_t)R.stride, (uintptr_t)R.sc, (uintptr_t)R.done,
            (uintptr_t)R.nblk_blas, (uintptr_t)g.block, (uintptr_t)g.swizzle, (uintptr_t)g.tps,
            (uintptr_t)g.tchunk, (uintptr_t)(g.nt + 1), (uintptr_t)g.rpt};
}

// Capture one plain CG iteration on R.s (the context's own stream) into a
// graph, unless the cached one matches.
static wl_status ensure_iteration_graph(CGRun &R) {
    wl_ctx *c = R.c;
    std::vector<uintptr_t> key = graph_key(R);
    if (c->cg_exec && key == c->cg_graph_key) return WL_OK;
    if (c->cg_exec) HIP_TRY(hipGraphExecDestroy(c->cg_exec));
    if (c->cg_graph) HIP_TRY(hipGraphDestroy(c->cg_graph));
    c->cg_exec = nullptr;
    c->cg_graph = nullptr;
    c->cg_graph_key.clear();
    HIP_TRY(hipStreamBeginCapture(R.s, hipStreamCaptureModeRelaxed));
    c->capturing = true;
    wl_status st = cg_iteration(R, false);
    c->capturing = false;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(R.s, &g);
    if (st) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return fail(WL_ERR_HIP, "stream capture failed: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&c->cg_exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return fail(WL_ERR_HIP, "graph instantiation failed: %s", hipGetErrorString(e));
    }
    c->cg_graph = g;
    c->cg_graph_key = key;
    return WL_OK;
}

// Fill R for a CG solve of context c (fields x, b; operator op) on stream s and
// make sure its workspace exists.
static wl_status cg_setup(wl_ctx *c, void *x, const void *b, int op, double kappa, int nrhs, const wl_solver_params &P,
                          hipStream_t s, CGRun &R) {
    const int subset = op == WL_OP_D ? WL_FULL : WL_EVEN;
    const int nh = subset == WL_FULL ? 2 : 1;
    std::memset(&R, 0, sizeof R);
    R.c = c;
    R.op = op;
    R.nrhs = nrhs;
    R.prec = P.prec;
    R.recon = P.recon;
    R.nh = nh;
    R.kappa = kappa;
    R.ru_restart = P.ru_restart < 0 ? (P.prec >= WL_F16N ? 1 : 0) : P.ru_restart;
    R.mu = P.mu;
    R.s = s;
    R.hb_lo = half_bytes(c, P.prec, nrhs);
    R.hb_hi = half_bytes(c, WL_F64, nrhs);
    if (overlap(x, R.hb_hi * nh, b, R.hb_hi * nh)) return fail(WL_ERR_ARG, "x and b overlap");
    R.x = x;
    R.b = b;
    R.stride = part_stride_for(c, nrhs);
    const size_t flo = R.hb_lo * nh, fhi = R.hb_hi * nh;
    wl_status st;
    // both link formats exist before anything is enqueued (building one synchronises
    // the device, which a graph capture of the iteration must not do)
    const void *lk;
    size_t sl;
    if ((st = get_links(c, WL_F64, 18, &lk, &sl)) || (st = get_links(c, P.prec, P.recon, &lk, &sl))) return st;
    if ((st = ensure_buf(c, S_R, flo)) || (st = ensure_buf(c, S_P, flo)) || (st = ensure_buf(c, S_Q, flo)) ||
        (st = ensure_buf(c, S_S, flo)) || (st = ensure_buf(c, S_TMP, R.hb_lo)) || (st = ensure_buf(c, S_RHI, fhi)) ||
        (st = ensure_buf(c, S_THI, fhi)) || (st = ensure_buf(c, S_TMPHI, R.hb_hi)) ||
        (st = ensure_buf(c, S_PARTIALS, sizeof(double) * 2 * nrhs * R.stride)) ||
        (st = ensure_buf(c, S_SCAL, std::max<size_t>(sizeof(CGScalars) * nrhs, 64 * sizeof(double) * 2))) ||
        (st = ensure_buf(c, S_BNORM, sizeof(double) * 2 * nrhs)) || (st = ensure_buf(c, S_FLAG, 64)) ||
        (st = ensure_pinned(c, sizeof(CGScalars) * nrhs + 64)))
        return st;
    R.r = c->buf[S_R];
    R.p = c->buf[S_P];
    R.q = c->buf[S_Q];
    R.sv = c->buf[S_S];
    R.tmp = c->buf[S_TMP];
    R.rhi = c->buf[S_RHI];
    R.thi = c->buf[S_THI];
    R.tmphi = c->buf[S_TMPHI];
    R.partials = (double *)c->buf[S_PARTIALS];
    R.sc = (CGScalars *)c->buf[S_SCAL];
    R.bnorm2 = (double *)c->buf[S_BNORM];
    R.done = (int *)c->buf[S_FLAG];
    R.nblk_blas = blas_blocks(c->Vh * (long)nrhs) * nh;
    if (P.prec == WL_F64) {
        R.r = R.rhi;  // FP64 CG iterates directly on the FP64 residual
    } else {
        R.hb_xlo = half_bytes(c, WL_F32, nrhs);
        if ((st = ensure_buf(c, S_XLO, R.hb_xlo * nh))) return st;
        R.xlo = c->buf[S_XLO];
        VecArgs z = vec_args(c, WL_F32, nrhs);
        set_vec(z, 0, R.xlo, R.hb_xlo);
        HIP_TRY(blas_zero(WL_F32, z, nh, s));
    }
    return WL_OK;
}

extern "C" wl_status wl_cg_solve(wl_ctx *c, void *x, const void *b, wl_op op, double kappa, int nrhs,
                                 const wl_solver_params *params, wl_solver_info *info, void *stream) {
    g_err.clear();
    const auto t0 = std::chrono::steady_clock::now();
    if (op != WL_OP_D && op != WL_OP_DHAT) return fail(WL_ERR_ARG, "bad operator %d", (int)op);
    const int subset = op == WL_OP_D ? WL_FULL : WL_EVEN;
    wl_status st = check_field_args(c, subset, WL_F64, nrhs);
    if (st) return st;
    wl_solver_params P;
    wl_solver_params_default(&P);
    if (params) P = *params;
    if (!prec_ok(P.prec)) return fail(WL_ERR_ARG, "bad inner precision %d", (int)P.prec);
    if (!recon_ok(P.prec, P.recon)) return fail(WL_ERR_UNSUPPORTED, "prec %d with recon %d not supported", P.prec, P.recon);
    if (!(P.tol >= 0.0) || !std::isfinite(kappa) || !std::isfinite(P.mu)) return fail(WL_ERR_ARG, "bad tolerance, kappa or mu");
    if (P.maxiter < 0 || P.check_every < 1 || P.max_restarts < 0) return fail(WL_ERR_ARG, "bad iteration limits");
    if (!x || !b || !aligned16(x) || !aligned16(b)) return fail(WL_ERR_ARG, "null or misaligned field pointer");
    CGRun R;
    hipStream_t run_stream = (hipStream_t)stream;
    const bool graph = P.use_graph != 0;
    if (graph) {
        // capture needs a stream other than the null stream: run the solve on the
        // context's own stream, ordered after the caller's work and before its next
        if (!c->own_stream) {
            HIP_TRY(hipStreamCreateWithFlags(&c->own_stream, hipStreamNonBlocking));
            HIP_TRY(hipEventCreateWithFlags(&c->handoff[0], hipEventDisableTiming));
            HIP_TRY(hipEventCreateWithFlags(&c->handoff[1], hipEventDisableTiming));
        }
        HIP_TRY(hipEventRecord(c->handoff[0], (hipStream_t)stream));
        HIP_TRY(hipStreamWaitEvent(c->own_stream, c->handoff[0], 0));
        run_stream = c->own_stream;
    }
    if ((st = cg_setup(c, x, b, op, kappa, nrhs, P, run_stream, R))) return st;
    const int nh = R.nh;
    const bool mixed = P.prec != WL_F64;

    // ||b||^2 per rhs
    {
        VecArgs v = vec_args(c, WL_F64, nrhs);
        set_vec(v, 0, b, R.hb_hi);
        v.partials = R.partials;
        v.part_stride = R.stride;
        HIP_TRY(blas_norm2(WL_F64, v, nh, R.s));
        HIP_TRY(reduce_partials(R.partials, R.stride, R.nblk_blas, nrhs, R.bnorm2, R.s));
    }
    std::vector<CGScalars> hsc(nrhs);
    std::vector<int> total_iters(nrhs, 0), reliable(nrhs, 0);
    int restarts = 0;
    int remaining = P.maxiter;
    wl_status result = WL_OK;
    std::vector<double> true_rel(nrhs, 0.0), iter_rel(nrhs, 0.0);
    std::vector<double> hb2(nrhs);
    HIP_TRY(hipMemcpyAsync(hb2.data(), R.bnorm2, sizeof(double) * nrhs, hipMemcpyDeviceToHost, R.s));
    for (;;) {
        // (re)start from the FP64 residual of the current x
        st = true_residual(R);
        if (st) return st;
        HIP_TRY(cg_init(R.sc, nrhs, R.partials, R.stride, R.nblk_blas, R.bnorm2, P.tol, remaining, R.done, R.s));
        st = load_residual(R);
        if (st) return st;
        int since_reliable = 0, k = 0;
        // Iterations are enqueued in blocks between host reads of the device
        // scalars.  Near convergence the block is sized from the observed decay
        // of ||r||^2 (with a margin), so that few or no iterations are enqueued
        // after the last one that does work (those launches exit at once).  In
        // mixed precision the same decay rate predicts the iteration at which
        // ||r|| will have dropped by reliable_delta, and the FP64 refresh is
        // scheduled there.
        // in mixed precision the first block is short, so that the decay rate (and with
        // it the first refresh) is known before the residual has fallen far
        int block = std::max(1, std::min(mixed ? std::min(4, P.check_every) : P.check_every, remaining));
        int ru_in = P.reliable_every > 0 ? P.reliable_every : INT32_MAX;  // iterations until the next refresh
        std::vector<double> prev_rho(nrhs, -1.0);
        std::vector<int> prev_it(nrhs, 0);
        ++c->timing_cycle;
        for (;;) {
            for (int j = 0; j < block; ++j, ++k) {
                bool ru = false;
                if (mixed && ++since_reliable >= ru_in) {
                    ru = true;
                    since_reliable = 0;
                    ru_in = P.reliable_every > 0 ? P.reliable_every : INT32_MAX;
                    for (int r = 0; r < nrhs; ++r) reliable[r]++;
                }
                c->timing_iter = k;
                if (graph && !ru) {
                    st = ensure_iteration_graph(R);
                    if (st) return st;
                    HIP_TRY(hipGraphLaunch(c->cg_exec, R.s));
                } else {
                    st = cg_iteration(R, ru);
                }
                c->timing_iter = -1;
                if (st) return st;
            }
            HIP_TRY(hipMemcpyAsync(c->host_pinned, R.sc, sizeof(CGScalars) * nrhs, hipMemcpyDeviceToHost, R.s));
            HIP_TRY(hipStreamSynchronize(R.s));
            std::memcpy(hsc.data(), c->host_pinned, sizeof(CGScalars) * nrhs);
            bool any = false;
            int next = 1;
            int ru_pred = INT32_MAX;
            for (int r = 0; r < nrhs; ++r) {
                const CGScalars &h = hsc[r];
                any |= h.active != 0;
                if (!h.active) continue;
                int est = P.check_every;
                if (prev_rho[r] > 0.0 && h.rho < prev_rho[r] && h.iter > prev_it[r]) {
                    const double rate = std::log(h.rho / prev_rho[r]) / (h.iter - prev_it[r]);  // < 0
                    if (h.target > 0.0) {
                        const double left = std::log(h.target / h.rho) / rate;
                        if (std::isfinite(left)) est = (int)std::floor(0.8 * left);
                    }
                    if (mixed) {
                        const double drop = P.reliable_delta * P.reliable_delta * h.rho_max;
                        const double until = h.rho <= drop ? 0.0 : std::log(drop / h.rho) / rate;
                        if (std::isfinite(until)) ru_pred = std::min(ru_pred, std::max(1, (int)std::ceil(until)));
                    }
                } else if (mixed && h.rho < P.reliable_delta * P.reliable_delta * h.rho_max) {
                    ru_pred = 1;
                }
                prev_rho[r] = h.rho;
                prev_it[r] = h.iter;
                next = std::max(next, std::min(est, P.check_every));
            }
            if (!any) break;
            block = std::max(1, next);
            if (mixed && ru_pred != INT32_MAX) {
                // refresh at the predicted drop (counted from now), or at the fixed cadence
                const int fixed_left = (P.reliable_every > 0 ? P.reliable_every : INT32_MAX) - since_reliable;
                ru_in = since_reliable + std::max(1, std::min(ru_pred, fixed_left));
            }
        }
        int maxit = 0;
        bool breakdown = false;
        for (int r = 0; r < nrhs; ++r) {
            total_iters[r] += hsc[r].iter;
            maxit = std::max(maxit, hsc[r].iter);
            iter_rel[r] = hb2[r] > 0 ? std::sqrt(hsc[r].rho / hb2[r]) : 0.0;
            breakdown |= hsc[r].status == WL_BREAKDOWN;
        }
        remaining -= maxit;
        if (c->timing) {
            // launches of iterations past the last one that ran exited at once: drop them
            auto &t = c->timed;
            t.erase(std::remove_if(t.begin(), t.end(),
                                   [&](const wl_ctx::TimedLaunch &x) {
                                       return x.cycle == c->timing_cycle && x.iter >= maxit;
                                   }),
                    t.end());
        }
        // FP64 true residual of the result
        st = true_residual(R);
        if (st) return st;
        std::vector<double> rr(nrhs);
        HIP_TRY(reduce_partials(R.partials, R.stride, R.nblk_blas, nrhs, R.bnorm2 + nrhs, R.s));
        HIP_TRY(hipMemcpyAsync(rr.data(), R.bnorm2 + nrhs, sizeof(double) * nrhs, hipMemcpyDeviceToHost, R.s));
        HIP_TRY(hipStreamSynchronize(R.s));
        bool all_ok = true;
        for (int r = 0; r < nrhs; ++r) {
            true_rel[r] = hb2[r] > 0 ? std::sqrt(rr[r] / hb2[r]) : 0.0;
            if (!(true_rel[r] <= P.tol)) all_ok = false;
        }
        if (breakdown) {
            result = WL_BREAKDOWN;
            break;
        }
        if (all_ok) {
            result = WL_OK;
            break;
        }
        if (remaining <= 0 || restarts >= P.max_restarts) {
            result = WL_NOT_CONVERGED;
            break;
        }
        ++restarts;
    }
    if (graph) {
        HIP_TRY(hipEventRecord(c->handoff[1], R.s));
        HIP_TRY(hipStreamWaitEvent((hipStream_t)stream, c->handoff[1], 0));
    }
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (info)
        for (int r = 0; r < nrhs; ++r) {
            info[r].iters = total_iters[r];
            info[r].restarts = restarts;
            info[r].reliable_updates = reliable[r];
            info[r].rel_resid = iter_rel[r];
            info[r].true_rel_resid = true_rel[r];
            info[r].seconds = secs;
        }
    if (result == WL_BREAKDOWN) fail(WL_BREAKDOWN, "CG breakdown (NaN/Inf or non-positive <p, A p>)");
    else if (result == WL_NOT_CONVERGED) fail(WL_NOT_CONVERGED, "CG did not reach the tolerance");
    return result;
}

// ------------------------------------------------------------------ batch of systems
// Several contexts (lattices of any size on this device) whose hopping-term
// launches are merged into one persistent launch per operator stage.
struct wl_batch {
    std::vector<wl_ctx *> ctx;
    int device = 0;
    hipStream_t s = nullptr;              // own non-blocking stream (graph capture)
    hipEvent_t handoff[2] = {nullptr, nullptr};
    int nwg = 0, block = 256, nt = -1;    // persistent workgroups, threads per tile, non-temporal
    int tps = 1;                          // threads per point (2: FP64 / FP32 storage only)
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<uintptr_t> key;
    bool timing = false, capturing = false;
    std::vector<std::array<hipEvent_t, 2>> timed;  // persistent launches while timing
    std::vector<hipEvent_t> pool;
    size_t pool_used = 0;
};

extern "C" wl_status wl_batch_create(wl_ctx *const *ctxs, int nsys, wl_batch **out) {
    g_err.clear();
    if (!ctxs || !out) return fail(WL_ERR_ARG, "null argument");
    *out = nullptr;
    if (nsys < 1 || nsys > BATCH_MAX) return fail(WL_ERR_ARG, "nsys %d not in 1..%d", nsys, BATCH_MAX);
    for (int k = 0; k < nsys; ++k) {
        if (!ctxs[k]) return fail(WL_ERR_ARG, "null context %d", k);
        if (ctxs[k]->device != ctxs[0]->device) return fail(WL_ERR_ARG, "contexts on different devices");
        for (int j = 0; j < k; ++j)
            if (ctxs[j] == ctxs[k]) return fail(WL_ERR_ARG, "context %d given twice", k);
    }
    wl_batch *B = new wl_batch();
    B->ctx.assign(ctxs, ctxs + nsys);
    B->device = ctxs[0]->device;
    int cus = 0;
    hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, B->device);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&B->s, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&B->handoff[0], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&B->handoff[1], hipEventDisableTiming);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        wl_batch_destroy(B);
        return fail(WL_ERR_HIP, "batch set-up: %s", hipGetErrorString(e));
    }
    // three 256-thread workgroups per compute unit stay resident with the FP32
    // hopping kernel's register use (138 VGPRs); a multiple of 8 so every XCD
    // gets the same number
    B->nwg = std::max(8, (cus * 3 + 7) / 8 * 8);
    *out = B;
    return WL_OK;
}

extern "C" wl_status wl_batch_destroy(wl_batch *B) {
    if (!B) return WL_OK;
    (void)hipDeviceSynchronize();
    if (B->exec) (void)hipGraphExecDestroy(B->exec);
    if (B->graph) (void)hipGraphDestroy(B->graph);
    for (hipEvent_t e : B->pool) (void)hipEventDestroy(e);
    for (hipEvent_t e : B->handoff)
        if (e) (void)hipEventDestroy(e);
    if (B->s) (void)hipStreamDestroy(B->s);
    delete B;
    return WL_OK;
}

// why a launch shape is not accepted, or null (also applied to autotuner cache entries)
static const char *launch_problem(int block, int tps, int nt, int rpt) {
    if (block < 64 || block > 256 || block % 64) return "block not in {64, 128, 192, 256}";
    if (tps != 1 && tps != 2) return "tps not in {1, 2}";
    if (nt < -1 || nt > 1) return "nt not in {-1, 0, 1}";
    if (rpt < 1 || rpt > 4) return "rpt not in 1..4";
    if (rpt > 1 && tps != 1) return "rpt > 1 needs tps = 1";
    return nullptr;
}

static const char *batch_launch_problem(int workgroups, int block, int nt, int tps) {
    if (workgroups != 0 && (workgroups < 8 || workgroups % 8 || workgroups > 65536))
        return "workgroups not 0 or a multiple of 8 in 8..65536";
    if (block < 64 || block > 256 || block % 64) return "block not in {64, 128, 192, 256}";
    if (nt < -1 || nt > 1) return "nt not in {-1, 0, 1}";
    if (tps != 1 && tps != 2) return "tps not in {1, 2}";
    return nullptr;
}

extern "C" wl_status wl_batch_set_launch(wl_batch *B, int workgroups, int block, int nt, int tps) {
    g_err.clear();
    if (!B) return fail(WL_ERR_ARG, "null batch");
    if (const char *why = batch_launch_problem(workgroups, block, nt, tps))
        return fail(WL_ERR_ARG, "batch launch (workgroups %d, block %d, nt %d, tps %d): %s", workgroups, block, nt,
                    tps, why);
    B->nwg = workgroups;
    B->block = block;
    B->nt = nt;
    B->tps = tps;
    return WL_OK;
}

extern "C" wl_status wl_batch_get_launch(const wl_batch *B, int *workgroups, int *block, int *nt, int *tps) {
    g_err.clear();
    if (!B || !workgroups || !block || !nt || !tps) return fail(WL_ERR_ARG, "null argument");
    *workgroups = B->nwg;
    *block = B->block;
    *nt = B->nt;
    *tps = B->tps;
    return WL_OK;
}

extern "C" wl_status wl_batch_timing_enable(wl_batch *B, int enable) {
    g_err.clear();
    if (!B) return fail(WL_ERR_ARG, "null batch");
    HIP_TRY(hipDeviceSynchronize());
    B->timed.clear();
    B->pool_used = 0;
    B->timing = enable != 0;
    return WL_OK;
}

extern "C" wl_status wl_batch_timing_read(wl_batch *B, int *count, double *total_ms) {
    g_err.clear();
    if (!B || !count || !total_ms) return fail(WL_ERR_ARG, "null argument");
    double ms = 0.0;
    for (auto &t : B->timed) {
        HIP_TRY(hipEventSynchronize(t[1]));
        float m = 0.f;
        HIP_TRY(hipEventElapsedTime(&m, t[0], t[1]));
        ms += m;
    }
    *count = (int)B->timed.size();
    *total_ms = ms;
    return WL_OK;
}

// out_k = M_k in_k (M_k^+ if dag) for every system k, one persistent launch per
// stage of the operator: D is one stage, D_hat two (odd hop into tmp_k, then the
// even hop with the epilogue).  With partials, ||out_k||^2 partials per rhs go
// to partials[k] (stride[k]) and nblk[k] receives their count.  flags[k]: the
// active count of system k's solver (tiles of a system whose count is 0 are
// skipped), or null.  With cg_sc (dag, partials set): the last stage does not store
// M_k^+ in_k but updates out_k = r_k -= alpha_k M_k^+ in_k in place, alpha_k per rhs
// from cg_sc[k], and the partials are those of ||r_k||^2.
static wl_status batch_apply(wl_batch *B, int op, bool dag, const double *kappa, int prec, int recon, int nrhs,
                             void *const *out, const void *const *in, void *const *tmp, double *const *partials,
                             const long *stride, int *const *flags, long *nblk, hipStream_t s, double mu = 0.0,
                             const CGScalars *const *cg_sc = nullptr) {
    const int n = (int)B->ctx.size();
    const int nst = op == WL_OP_D ? 1 : 2;
    const int tps = (prec == WL_F64 || prec == WL_F32) && B->tps == 2 ? 2 : 1;
    if (cg_sc && (!dag || !partials)) return fail(WL_ERR_ARG, "the residual update needs M^+ and norm partials");
    if (B->nwg == 0) {
        // one launch per system and stage, each with its context's own launch shape
        for (int k = 0; k < n; ++k) {
            wl_ctx *c = B->ctx[k];
            void *tk = tmp ? tmp[k] : nullptr;
            const int *fk = flags ? flags[k] : nullptr;
            long nb = 0;
            wl_status st = cg_sc ? apply_mdag_update_r(c, op, kappa[k], prec, recon, nrhs, out[k], in[k], tk,
                                                       partials[k], stride[k], fk, s, &nb, mu, cg_sc[k])
                                 : apply_m(c, op, dag, kappa[k], prec, recon, nrhs, out[k], in[k], tk,
                                           partials ? partials[k] : nullptr, partials ? stride[k] : 0, fk, s,
                                           &nb, mu);
            if (st) return st;
            if (nblk) nblk[k] = nb;
        }
        return WL_OK;
    }
    for (int stage = 0; stage < nst; ++stage) {
        BatchArgs A;
        std::memset(&A, 0, sizeof A);
        A.nsys = n;
        long tiles = 0;
        double ws = 0.0;
        const bool last = stage == nst - 1;
        const int epi = last ? (EPI_XPAY | (partials ? EPI_NORM : 0) | (cg_sc ? EPI_CGR : 0)) : 0;
        for (int k = 0; k < n; ++k) {
            wl_ctx *c = B->ctx[k];
            HopArgs &h = A.sys[k];
            int np = 1;
            const int *flag = flags ? flags[k] : nullptr;
            double *pk = partials ? partials[k] : nullptr;
            const long sk = partials ? stride[k] : 0;
            wl_status st;
            // twisted mass as in apply_m
            const double nu = (dag ? -2.0 : 2.0) * kappa[k] * mu;
            if (op == WL_OP_D)
                st = fill_hop_args(c, prec, recon, out[k], in[k], in[k], WL_FULL, nrhs, 1.0, -kappa[k], pk, sk, flag, h,
                                   &np, nu, 0.0);
            else if (stage == 0)
                st = fill_hop_args(c, prec, recon, tmp[k], in[k], nullptr, WL_ODD, nrhs, 0.0, 1.0 / (1.0 + nu * nu),
                                   nullptr, 0, flag, h, &np, 0.0, -nu);
            else
                st = fill_hop_args(c, prec, recon, out[k], tmp[k], in[k], WL_EVEN, nrhs, 1.0, -kappa[k] * kappa[k], pk,
                                   sk, flag, h, &np, nu, 0.0);
            if (st) return st;
            if (epi & EPI_CGR) set_cg_residual(c, prec, nrhs, op == WL_OP_D ? WL_FULL : WL_EVEN, out[k], cg_sc[k], h);
            A.per_par[k] = hop_blocks(h.npts, B->block, tps);
            A.start[k] = tiles;
            tiles += A.per_par[k] * np;
            if (nblk && last) nblk[k] = A.per_par[k] * np;
            ws += 8.0 * (double)h.slab_bytes +
                  (double)padded(h.npts) * np * spinor_point_bytes(prec) * ((epi & EPI_XPAY) ? 3 : 2);
        }
        A.start[n] = tiles;
        A.ntiles = tiles;
        const bool nt = B->nt >= 0 ? B->nt != 0 : ws > 200e6;
        hipEvent_t *ev = nullptr;
        if (B->timing && !B->capturing && B->timed.size() < (1u << 16)) {
            if (B->pool_used + 2 > B->pool.size())
                for (int k = 0; k < 256; ++k) {
                    hipEvent_t e;
                    HIP_TRY(hipEventCreate(&e));
                    B->pool.push_back(e);
                }
            B->timed.push_back({B->pool[B->pool_used], B->pool[B->pool_used + 1]});
            B->pool_used += 2;
            ev = B->timed.back().data();
            HIP_TRY(hipEventRecord(ev[0], s));
        }
        HIP_TRY(launch_hop_batch(prec, recon, dag, epi, nt, tps, A, B->nwg, B->block, s));
        if (ev) HIP_TRY(hipEventRecord(ev[1], s));
    }
    return WL_OK;
}

static wl_status batch_check(wl_batch *B, int prec, int recon, int nrhs, int subset) {
    if (!B) return fail(WL_ERR_ARG, "null batch");
    if (!prec_ok(prec)) return fail(WL_ERR_ARG, "bad precision %d", prec);
    if (!recon_ok(prec, recon)) return fail(WL_ERR_UNSUPPORTED, "prec %d with recon %d not supported", prec, recon);
    if (nrhs < 1 || nrhs > 64) return fail(WL_ERR_ARG, "nrhs %d not in 1..64", nrhs);
    for (wl_ctx *c : B->ctx) {
        wl_status st = check_field_args(c, subset, prec, nrhs);
        if (st) return st;
    }
    return WL_OK;
}

extern "C" wl_status wl_batch_dirac_apply(wl_batch *B, void *const *out, const void *const *in, wl_op op, int dagger,
                                          const double *kappa, wl_prec prec, int recon, int nrhs, void *stream) {
    g_err.clear();
    if (op != WL_OP_D && op != WL_OP_DHAT) return fail(WL_ERR_ARG, "bad operator %d", (int)op);
    wl_status st = batch_check(B, prec, recon, nrhs, op == WL_OP_D ? WL_FULL : WL_EVEN);
    if (st) return st;
    if (!out || !in || !kappa) return fail(WL_ERR_ARG, "null argument");
    const int n = (int)B->ctx.size();
    std::vector<void *> tmp(n, nullptr);
    for (int k = 0; k < n; ++k) {
        wl_ctx *c = B->ctx[k];
        if (!out[k] || !in[k] || !aligned16(out[k]) || !aligned16(in[k]))
            return fail(WL_ERR_ARG, "null or misaligned field pointer of system %d", k);
        if (!std::isfinite(kappa[k])) return fail(WL_ERR_ARG, "non-finite kappa of system %d", k);
        const size_t hb = half_bytes(c, prec, nrhs), bytes = hb * (op == WL_OP_D ? 2 : 1);
        if (overlap(out[k], bytes, in[k], bytes)) return fail(WL_ERR_ARG, "out and in of system %d overlap", k);
        if (op == WL_OP_DHAT) {
            if ((st = ensure_buf(c, S_TMP_OP, hb))) return st;
            tmp[k] = c->buf[S_TMP_OP];
        }
    }
    return batch_apply(B, op, dagger != 0, kappa, prec, recon, nrhs, out, in, tmp.data(), nullptr, nullptr, nullptr,
                       nullptr, (hipStream_t)stream);
}

// One CG iteration of every system in lockstep: the four (two for D) hopping
// stages are persistent launches over all systems, the scalar and vector steps
// are per system.  ru[k]: FP64 refresh of system k in this iteration.
static wl_status batch_iteration(wl_batch *B, std::vector<CGRun> &R, const std::vector<char> &ru) {
    const int n = (int)R.size();
    const CGRun &R0 = R[0];
    std::vector<void *> q(n), p(n), sv(n), tmp(n);
    std::vector<double *> part(n);
    std::vector<long> stride(n), nblk(n);
    std::vector<int *> flags(n);
    std::vector<double> kap(n);
    for (int k = 0; k < n; ++k) {
        q[k] = R[k].q;
        p[k] = R[k].p;
        sv[k] = R[k].sv;
        tmp[k] = R[k].tmp;
        part[k] = R[k].partials;
        stride[k] = R[k].stride;
        flags[k] = R[k].done;
        kap[k] = R[k].kappa;
    }
    wl_status st = batch_apply(B, R0.op, false, kap.data(), R0.prec, R0.recon, R0.nrhs, q.data(),
                               (const void *const *)p.data(), tmp.data(), part.data(), stride.data(), flags.data(),
                               nblk.data(), R0.s, R0.mu);
    if (st) return st;
    for (int k = 0; k < n; ++k)
        HIP_TRY(cg_alpha(R[k].sc, R[k].nrhs, R[k].partials, R[k].stride, nblk[k], R[k].done, R[k].s));
    bool fused = true;
    for (int k = 0; k < n; ++k) {
        fused = fused && !ru[k];
        // per-system launches take the fused form only with one rhs per thread
        const LaunchCfg &g = R[k].c->cfg[R[k].prec];
        if (B->nwg == 0) fused = fused && effective_rpt(g, R[k].nrhs, effective_tps(R[k].prec, g)) == 1;
    }
    if (fused) {
        // as in the single-system iteration: the last stage updates r_k in place
        // (r -= alpha A p, ||r||^2), then beta and x += alpha p, p = r + beta p
        std::vector<void *> r(n);
        std::vector<const CGScalars *> sc(n);
        for (int k = 0; k < n; ++k) {
            r[k] = R[k].r;
            sc[k] = R[k].sc;
        }
        st = batch_apply(B, R0.op, true, kap.data(), R0.prec, R0.recon, R0.nrhs, r.data(),
                         (const void *const *)q.data(), tmp.data(), part.data(), stride.data(), flags.data(),
                         nblk.data(), R0.s, R0.mu, sc.data());
        if (st) return st;
        for (int k = 0; k < n; ++k) {
            HIP_TRY(cg_beta(R[k].sc, R[k].nrhs, R[k].partials, R[k].stride, nblk[k], R[k].done, 0, R[k].s));
            VecArgs u = vec_args(R[k].c, R[k].prec, R[k].nrhs);
            set_vec(u, 0, R[k].xlo ? R[k].xlo : R[k].x, R[k].xlo ? R[k].hb_xlo : R[k].hb_hi);
            set_vec(u, 1, R[k].p, R[k].hb_lo);
            set_vec(u, 2, R[k].r, R[k].hb_lo);
            u.sc = R[k].sc;
            u.flag = nullptr;  // must also run after the system's final step
            HIP_TRY(cg_update_xp(R[k].prec, R[k].xlo ? WL_F32 : WL_F64, u, R[k].nh, R[k].s));
        }
        return WL_OK;
    }
    st = batch_apply(B, R0.op, true, kap.data(), R0.prec, R0.recon, R0.nrhs, sv.data(), (const void *const *)q.data(),
                     tmp.data(), nullptr, nullptr, flags.data(), nullptr, R0.s, R0.mu);
    if (st) return st;
    for (int k = 0; k < n; ++k)
        if ((st = cg_finish_iteration(R[k], ru[k] != 0))) return st;
    return WL_OK;
}

static wl_status ensure_batch_graph(wl_batch *B, std::vector<CGRun> &R) {
    std::vector<uintptr_t> key{(uintptr_t)B->nwg, (uintptr_t)B->block, (uintptr_t)(B->nt + 1), (uintptr_t)B->tps};
    for (auto &r : R) {
        std::vector<uintptr_t> k = graph_key(r);
        key.insert(key.end(), k.begin(), k.end());
    }
    if (B->exec && key == B->key) return WL_OK;
    if (B->exec) HIP_TRY(hipGraphExecDestroy(B->exec));
    if (B->graph) HIP_TRY(hipGraphDestroy(B->graph));
    B->exec = nullptr;
    B->graph = nullptr;
    B->key.clear();
    HIP_TRY(hipStreamBeginCapture(B->s, hipStreamCaptureModeRelaxed));
    B->capturing = true;
    for (auto &r : R) r.c->capturing = true;
    wl_status st = batch_iteration(B, R, std::vector<char>(R.size(), 0));
    B->capturing = false;
    for (auto &r : R) r.c->capturing = false;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(B->s, &g);
    if (st) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return fail(WL_ERR_HIP, "stream capture failed: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&B->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return fail(WL_ERR_HIP, "graph instantiation failed: %s", hipGetErrorString(e));
    }
    B->graph = g;
    B->key = key;
    return WL_OK;
}

extern "C" wl_status wl_batch_cg_solve(wl_batch *B, void *const *x, const void *const *b, wl_op op,
                                       const double *kappa, int nrhs, const wl_solver_params *params,
                                       wl_solver_info *info, void *stream) {
    g_err.clear();
    const auto t0 = std::chrono::steady_clock::now();
    if (op != WL_OP_D && op != WL_OP_DHAT) return fail(WL_ERR_ARG, "bad operator %d", (int)op);
    const int subset = op == WL_OP_D ? WL_FULL : WL_EVEN;
    wl_solver_params P;
    wl_solver_params_default(&P);
    if (params) P = *params;
    wl_status st = batch_check(B, WL_F64, 18, nrhs, subset);
    if (st) return st;
    if (!prec_ok(P.prec)) return fail(WL_ERR_ARG, "bad inner precision %d", (int)P.prec);
    if (!recon_ok(P.prec, P.recon)) return fail(WL_ERR_UNSUPPORTED, "prec %d with recon %d not supported", P.prec, P.recon);
    if (!(P.tol >= 0.0)) return fail(WL_ERR_ARG, "bad tolerance");
    if (P.maxiter < 0 || P.check_every < 1 || P.max_restarts < 0) return fail(WL_ERR_ARG, "bad iteration limits");
    if (!x || !b || !kappa) return fail(WL_ERR_ARG, "null argument");
    const int n = (int)B->ctx.size();
    for (int k = 0; k < n; ++k) {
        if (!x[k] || !b[k] || !aligned16(x[k]) || !aligned16(b[k]))
            return fail(WL_ERR_ARG, "null or misaligned field pointer of system %d", k);
        if (!std::isfinite(kappa[k])) return fail(WL_ERR_ARG, "non-finite kappa of system %d", k);
    }
    const bool graph = P.use_graph != 0;
    hipStream_t s = (hipStream_t)stream;
    if (graph) {
        HIP_TRY(hipEventRecord(B->handoff[0], (hipStream_t)stream));
        HIP_TRY(hipStreamWaitEvent(B->s, B->handoff[0], 0));
        s = B->s;
    }
    std::vector<CGRun> R(n);
    for (int k = 0; k < n; ++k)
        if ((st = cg_setup(B->ctx[k], x[k], b[k], op, kappa[k], nrhs, P, s, R[k]))) return st;
    const int nh = R[0].nh;
    const bool mixed = P.prec != WL_F64;
    // ||b||^2 per system and rhs
    std::vector<std::vector<double>> hb2(n, std::vector<double>(nrhs));
    for (int k = 0; k < n; ++k) {
        VecArgs v = vec_args(R[k].c, WL_F64, nrhs);
        set_vec(v, 0, b[k], R[k].hb_hi);
        v.partials = R[k].partials;
        v.part_stride = R[k].stride;
        HIP_TRY(blas_norm2(WL_F64, v, nh, s));
        HIP_TRY(reduce_partials(R[k].partials, R[k].stride, R[k].nblk_blas, nrhs, R[k].bnorm2, s));
        HIP_TRY(hipMemcpyAsync(hb2[k].data(), R[k].bnorm2, sizeof(double) * nrhs, hipMemcpyDeviceToHost, s));
    }
    HIP_TRY(hipStreamSynchronize(s));
    std::vector<std::vector<CGScalars>> hsc(n, std::vector<CGScalars>(nrhs));
    std::vector<std::vector<int>> total(n, std::vector<int>(nrhs, 0)), relu(n, std::vector<int>(nrhs, 0));
    std::vector<std::vector<double>> true_rel(n, std::vector<double>(nrhs, 0.0)),
        iter_rel(n, std::vector<double>(nrhs, 0.0));
    int restarts = 0, remaining = P.maxiter;
    wl_status result = WL_OK;
    const int ru_every = P.reliable_every > 0 ? P.reliable_every : INT32_MAX;
    for (;;) {
        for (int k = 0; k < n; ++k) {
            if ((st = true_residual(R[k]))) return st;
            HIP_TRY(cg_init(R[k].sc, nrhs, R[k].partials, R[k].stride, R[k].nblk_blas, R[k].bnorm2, P.tol, remaining,
                            R[k].done, s));
            if ((st = load_residual(R[k]))) return st;
        }
        // refresh schedule and host-check blocks as in wl_cg_solve, per system: a short
        // first block, then blocks and refreshes predicted from the observed decay
        std::vector<int> since(n, 0), ru_in(n, ru_every);
        std::vector<char> live(n, 1);
        std::vector<std::vector<double>> prev_rho(n, std::vector<double>(nrhs, -1.0));
        std::vector<std::vector<int>> prev_it(n, std::vector<int>(nrhs, 0));
        int block = std::max(1, std::min(mixed ? std::min(4, P.check_every) : P.check_every, remaining));
        for (;;) {
            for (int j = 0; j < block; ++j) {
                std::vector<char> ru(n, 0);
                bool any_ru = false;
                if (mixed)
                    for (int k = 0; k < n; ++k)
                        if (live[k] && ++since[k] >= ru_in[k]) {
                            ru[k] = 1;
                            any_ru = true;
                            since[k] = 0;
                            ru_in[k] = ru_every;
                            for (int r = 0; r < nrhs; ++r)
                                if (hsc[k][r].active || prev_rho[k][r] < 0.0) relu[k][r]++;
                        }
                if (graph && !any_ru) {
                    if ((st = ensure_batch_graph(B, R))) return st;
                    HIP_TRY(hipGraphLaunch(B->exec, s));
                } else if ((st = batch_iteration(B, R, ru))) {
                    return st;
                }
            }
            for (int k = 0; k < n; ++k)
                HIP_TRY(hipMemcpyAsync(R[k].c->host_pinned, R[k].sc, sizeof(CGScalars) * nrhs, hipMemcpyDeviceToHost,
                                       s));
            HIP_TRY(hipStreamSynchronize(s));
            bool any = false;
            int next = 1;
            for (int k = 0; k < n; ++k) {
                std::memcpy(hsc[k].data(), R[k].c->host_pinned, sizeof(CGScalars) * nrhs);
                int ru_pred = INT32_MAX;
                bool sys_live = false;
                for (int r = 0; r < nrhs; ++r) {
                    const CGScalars &h = hsc[k][r];
                    if (!h.active) continue;
                    sys_live = true;
                    int est = P.check_every;
                    if (prev_rho[k][r] > 0.0 && h.rho < prev_rho[k][r] && h.iter > prev_it[k][r]) {
                        const double rate = std::log(h.rho / prev_rho[k][r]) / (h.iter - prev_it[k][r]);
                        if (h.target > 0.0) {
                            const double left = std::log(h.target / h.rho) / rate;
                            if (std::isfinite(left)) est = (int)std::floor(0.8 * left);
                        }
                        if (mixed) {
                            const double drop = P.reliable_delta * P.reliable_delta * h.rho_max;
                            const double until = h.rho <= drop ? 0.0 : std::log(drop / h.rho) / rate;
                            if (std::isfinite(until)) ru_pred = std::min(ru_pred, std::max(1, (int)std::ceil(until)));
                        }
                    } else if (mixed && h.rho < P.reliable_delta * P.reliable_delta * h.rho_max) {
                        ru_pred = 1;
                    }
                    prev_rho[k][r] = h.rho;
                    prev_it[k][r] = h.iter;
                    next = std::max(next, std::min(est, P.check_every));
                }
                live[k] = sys_live;
                any |= sys_live;
                if (mixed && sys_live && ru_pred != INT32_MAX)
                    ru_in[k] = since[k] + std::max(1, std::min(ru_pred, ru_every - since[k]));
            }
            if (!any) break;
            block = std::max(1, next);
        }
        int maxit = 0;
        bool breakdown = false, all_ok = true;
        for (int k = 0; k < n; ++k) {
            for (int r = 0; r < nrhs; ++r) {
                total[k][r] += hsc[k][r].iter;
                maxit = std::max(maxit, hsc[k][r].iter);
                iter_rel[k][r] = hb2[k][r] > 0 ? std::sqrt(hsc[k][r].rho / hb2[k][r]) : 0.0;
                breakdown |= hsc[k][r].status == WL_BREAKDOWN;
            }
            if ((st = true_residual(R[k]))) return st;
            HIP_TRY(reduce_partials(R[k].partials, R[k].stride, R[k].nblk_blas, nrhs, R[k].bnorm2 + nrhs, s));
        }
        std::vector<std::vector<double>> rr(n, std::vector<double>(nrhs));
        for (int k = 0; k < n; ++k)
            HIP_TRY(hipMemcpyAsync(rr[k].data(), R[k].bnorm2 + nrhs, sizeof(double) * nrhs, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        remaining -= maxit;
        for (int k = 0; k < n; ++k)
            for (int r = 0; r < nrhs; ++r) {
                true_rel[k][r] = hb2[k][r] > 0 ? std::sqrt(rr[k][r] / hb2[k][r]) : 0.0;
                if (!(true_rel[k][r] <= P.tol)) all_ok = false;
            }
        if (breakdown) {
            result = WL_BREAKDOWN;
            break;
        }
        if (all_ok) break;
        if (remaining <= 0 || restarts >= P.max_restarts) {
            result = WL_NOT_CONVERGED;
            break;
        }
        ++restarts;
    }
    if (graph) {
        HIP_TRY(hipEventRecord(B->handoff[1], s));
        HIP_TRY(hipStreamWaitEvent((hipStream_t)stream, B->handoff[1], 0));
    }
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (info)
        for (int k = 0; k < n; ++k)
            for (int r = 0; r < nrhs; ++r) {
                wl_solver_info &o = info[k * nrhs + r];
                o = wl_solver_info{};
                o.iters = total[k][r];
                o.restarts = restarts;
                o.reliable_updates = relu[k][r];
                o.rel_resid = iter_rel[k][r];
                o.true_rel_resid = true_rel[k][r];
                o.seconds = secs;
            }
    if (result == WL_BREAKDOWN) fail(WL_BREAKDOWN, "CG breakdown (NaN/Inf or non-positive <p, A p>)");
    else if (result == WL_NOT_CONVERGED) fail(WL_NOT_CONVERGED, "batched CG did not reach the tolerance");
    return result;
}

// ------------------------------------------------------------------ autotuner
namespace {
std::string arch_name(int device) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return "unknown";
    std::string a = prop.gcnArchName;
    const size_t colon = a.find(':');
    return colon == std::string::npos ? a : a.substr(0, colon);
}

// In-process cache of tuned launches, keyed by a text key; optionally mirrored
// in a text file, one entry per line: "<key> | <values...>".
std::vector<std::pair<std::string, std::vector<double>>> g_tuned;

bool cache_lookup(const std::string &key, const char *path, std::vector<double> &vals) {
    for (auto &e : g_tuned)
        if (e.first == key) {
            vals = e.second;
            return true;
        }
    if (!path) return false;
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    char line[1024];
    bool found = false;
    while (std::fgets(line, sizeof line, f)) {
        std::string l(line);
        const size_t bar = l.find(" | ");
        if (bar == std::string::npos || l.substr(0, bar) != key) continue;
        std::vector<double> v;
        const char *q = l.c_str() + bar + 3;
        char *end = nullptr;
        for (;;) {
            const double d = std::strtod(q, &end);
            if (end == q) break;
            v.push_back(d);
            q = end;
        }
        if (!v.empty()) {
            vals = v;  // the last matching line wins
            found = true;
        }
    }
    std::fclose(f);
    if (found) g_tuned.push_back({key, vals});
    return found;
}

void cache_store(const std::string &key, const char *path, const std::vector<double> &vals) {
    bool replaced = false;
    for (auto &e : g_tuned)
        if (e.first == key) {
            e.second = vals;
            replaced = true;
        }
    if (!replaced) g_tuned.push_back({key, vals});
    if (!path) return;
    FILE *f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%s |", key.c_str());
    for (double v : vals) std::fprintf(f, " %.6g", v);
    std::fprintf(f, "\n");
    std::fclose(f);
}

// average time of `reps` launches of fn (after one warm-up), microseconds
template <typename F>
wl_status time_launches(F fn, int reps, hipStream_t s, double *us) {
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    wl_status st = fn();
    if (!st) {
        (void)hipEventRecord(e0, s);
        for (int k = 0; k < reps && !st; ++k) st = fn();
        (void)hipEventRecord(e1, s);
        (void)hipEventSynchronize(e1);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        *us = 1e3 * ms / reps;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return st;
}
}  // namespace

extern "C" wl_status wl_autotune(wl_ctx *c, wl_prec prec, int recon, int nrhs, const char *cache_path,
                                 wl_launch *chosen, double *best_us, int *from_cache) {
    g_err.clear();
    wl_status st = check_field_args(c, WL_FULL, prec, nrhs);
    if (st) return st;
    if (!recon_ok(prec, recon)) return fail(WL_ERR_UNSUPPORTED, "prec %d with recon %d not supported", prec, recon);
    char kb[256];
    std::snprintf(kb, sizeof kb, "hop %s %d %d %d %d prec %d recon %d nrhs %d", arch_name(c->device).c_str(),
                  c->dims[0], c->dims[1], c->dims[2], c->dims[3], (int)prec, recon, nrhs);
    const std::string key(kb);
    std::vector<double> vals;
    LaunchCfg best;
    double best_t = 0.0;
    int cached = 0;
    // a cache entry that is not a valid launch shape is ignored (and tuned again)
    if (cache_lookup(key, cache_path, vals) && vals.size() >= 7 &&
        !launch_problem((int)vals[0], (int)vals[2], (int)vals[4], (int)vals[5])) {
        best.block = (int)vals[0];
        best.swizzle = (int)vals[1];
        best.tps = (int)vals[2];
        best.tchunk = (int)vals[3];
        best.nt = (int)vals[4];
        best.rpt = (int)vals[5];
        best_t = vals[6];
        cached = 1;
    } else {
        // the solvers' launch: out = x - kappa H in over both parities, on scratch fields
        const size_t full = 2 * half_bytes(c, prec, nrhs);
        void *buf = nullptr;
        if (hipMalloc(&buf, 3 * full) != hipSuccess) {
            (void)hipGetLastError();
            return fail(WL_ERR_NOMEM, "autotune scratch of %zu bytes", 3 * full);
        }
        if (hipMemset(buf, 0, 3 * full) != hipSuccess) {
            (void)hipFree(buf);
            return fail(WL_ERR_HIP, "autotune scratch clear failed");
        }
        char *in = (char *)buf, *out = in + full, *x = out + full;
        const LaunchCfg saved = c->cfg[prec];
        const bool saved_timing = c->timing;
        c->timing = false;
        const bool two = prec == WL_F64 || prec == WL_F32;
        best_t = 1e30;
        for (int block : {64, 128, 256})
            for (int tps : {1, 2})
                for (int rpt : {1, 2, 3, 4})
                for (int swz : {0, 1})
                    for (int tch : {0, 4, WL_TCHUNK_AUTO})
                        for (int nt : {0, 1}) {
                            if (st) break;  // the first failure ends the sweep
                            if (tps == 2 && !two) continue;
                            if (rpt > 1 && (tps != 1 || nrhs % rpt)) continue;
                            if (tch > 0 && tch >= c->dims[3]) continue;
                            LaunchCfg g;
                            g.block = block;
                            g.tps = tps;
                            g.rpt = rpt;
                            g.swizzle = swz;
                            g.tchunk = tch;
                            g.nt = nt;
                            c->cfg[prec] = g;
                            double us = 0.0;
                            st = time_launches(
                                [&]() {
                                    return hop_core(c, prec, recon, false, EPI_XPAY, out, in, x, WL_FULL, nrhs, 1.0,
                                                    -0.1, nullptr, 0, nullptr, nullptr);
                                },
                                5, nullptr, &us);
                            if (st) break;
                            if (us < best_t) {
                                best_t = us;
                                best = g;
                            }
                        }
        c->cfg[prec] = saved;
        c->timing = saved_timing;
        (void)hipFree(buf);
        if (st) return st;
        cache_store(key, cache_path,
                    {(double)best.block, (double)best.swizzle, (double)best.tps, (double)best.tchunk, (double)best.nt,
                     (double)best.rpt, best_t});
    }
    c->cfg[prec] = best;
    if (chosen) {
        chosen->block = best.block;
        chosen->swizzle = best.swizzle;
        chosen->tps = best.tps;
        chosen->tchunk = best.tchunk;
        chosen->nt = best.nt;
        chosen->rpt = best.rpt;
    }
    if (best_us) *best_us = best_t;
    if (from_cache) *from_cache = cached;
    return WL_OK;
}

extern "C" wl_status wl_batch_autotune(wl_batch *B, wl_prec prec, int recon, int nrhs, const char *cache_path,
                                       int *workgroups, int *block, int *nt, int *tps, double *best_us,
                                       int *from_cache) {
    g_err.clear();
    wl_status st = batch_check(B, prec, recon, nrhs, WL_FULL);
    if (st) return st;
    const int n = (int)B->ctx.size();
    int cus = 0;
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, B->device));
    std::string key = "batch " + arch_name(B->device);
    for (wl_ctx *c : B->ctx)
        key += " " + std::to_string(c->dims[0]) + "x" + std::to_string(c->dims[1]) + "x" + std::to_string(c->dims[2]) +
               "x" + std::to_string(c->dims[3]);
    key += " prec " + std::to_string((int)prec) + " recon " + std::to_string(recon) + " nrhs " + std::to_string(nrhs);
    std::vector<double> vals;
    int bw = B->nwg, bb = B->block, bn = B->nt, bt = B->tps, cached = 0;
    double best_t = 0.0;
    if (cache_lookup(key, cache_path, vals) && vals.size() >= 5 &&
        !batch_launch_problem((int)vals[0], (int)vals[1], (int)vals[2], (int)vals[3])) {
        bw = (int)vals[0];
        bb = (int)vals[1];
        bn = (int)vals[2];
        bt = (int)vals[3];
        best_t = vals[4];
        cached = 1;
    } else {
        std::vector<void *> bufs(n, nullptr), outs(n), ins(n);
        std::vector<double> kap(n, 0.1);
        for (int k = 0; k < n && !st; ++k) {
            const size_t full = 2 * half_bytes(B->ctx[k], prec, nrhs);
            if (hipMalloc(&bufs[k], 2 * full) != hipSuccess || hipMemset(bufs[k], 0, 2 * full) != hipSuccess) {
                st = fail(WL_ERR_NOMEM, "autotune scratch of system %d", k);
                break;
            }
            ins[k] = bufs[k];
            outs[k] = (char *)bufs[k] + full;
        }
        const int sw = B->nwg, sb = B->block, sn = B->nt, st2 = B->tps;
        const bool two = prec == WL_F64 || prec == WL_F32;
        const bool saved_timing = B->timing;
        B->timing = false;
        best_t = 1e30;
        // first candidate: one launch per system with each context's own shape
        B->nwg = 0;
        {
            double us = 0.0;
            st = time_launches(
                [&]() {
                    return batch_apply(B, WL_OP_D, false, kap.data(), prec, recon, nrhs, outs.data(),
                                       (const void *const *)ins.data(), nullptr, nullptr, nullptr, nullptr, nullptr,
                                       nullptr);
                },
                5, nullptr, &us);
            if (!st) {
                best_t = us;
                bw = 0;
                bb = sb;
                bn = sn;
                bt = st2;
            }
        }
        for (int tpv : {1, 2})
        for (int per_cu : {1, 2, 3, 4, 6, 8})
            for (int blk : {64, 128, 256})
                for (int ntv : {0, 1}) {
                    if (st) break;
                    if (tpv == 2 && !two) continue;
                    B->nwg = std::max(8, (cus * per_cu * 256 / blk + 7) / 8 * 8);
                    B->block = blk;
                    B->nt = ntv;
                    B->tps = tpv;
                    double us = 0.0;
                    st = time_launches(
                        [&]() {
                            return batch_apply(B, WL_OP_D, false, kap.data(), prec, recon, nrhs, outs.data(),
                                               (const void *const *)ins.data(), nullptr, nullptr, nullptr, nullptr,
                                               nullptr, nullptr);
                        },
                        5, nullptr, &us);
                    if (!st && us < best_t) {
                        best_t = us;
                        bw = B->nwg;
                        bb = blk;
                        bn = ntv;
                        bt = tpv;
                    }
                }
        B->nwg = sw;
        B->block = sb;
        B->nt = sn;
        B->tps = st2;
        B->timing = saved_timing;
        for (void *p : bufs)
            if (p) (void)hipFree(p);
        if (st) return st;
        cache_store(key, cache_path, {(double)bw, (double)bb, (double)bn, (double)bt, best_t});
    }
    B->nwg = bw;
    B->block = bb;
    B->nt = bn;
    B->tps = bt;
    if (workgroups) *workgroups = bw;
    if (block) *block = bb;
    if (nt) *nt = bn;
    if (tps) *tps = bt;
    if (best_us) *best_us = best_t;
    if (from_cache) *from_cache = cached;
    return WL_OK;
}

// ------------------------------------------------------------------ incremental EigCG
namespace {
using cd = std::complex<double>;

// Eigenvalues (ascending) and orthonormal eigenvectors (column k of the
// row-major n x n array v) of a real symmetric matrix, cyclic Jacobi rotations.
void sym_eig(int n, std::vector<double> a, std::vector<double> &w, std::vector<double> &v) {
    v.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) v[(size_t)i * n + i] = 1.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                const double x = a[(size_t)i * n + j] * a[(size_t)i * n + j];
                tot += x;
                if (i != j) off += x;
            }
        if (off <= 1e-30 * tot) break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                const double apq = a[(size_t)p * n + q];
                if (std::fabs(apq) < 1e-300) continue;
                const double theta = (a[(size_t)q * n + q] - a[(size_t)p * n + p]) / (2.0 * apq);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), sn = t * c;
                for (int k = 0; k < n; ++k) {  // columns p, q
                    const double akp = a[(size_t)k * n + p], akq = a[(size_t)k * n + q];
                    a[(size_t)k * n + p] = c * akp - sn * akq;
                    a[(size_t)k * n + q] = sn * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {  // rows p, q
                    const double apk = a[(size_t)p * n + k], aqk = a[(size_t)q * n + k];
                    a[(size_t)p * n + k] = c * apk - sn * aqk;
                    a[(size_t)q * n + k] = sn * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    const double vkp = v[(size_t)k * n + p], vkq = v[(size_t)k * n + q];
                    v[(size_t)k * n + p] = c * vkp - sn * vkq;
                    v[(size_t)k * n + q] = sn * vkp + c * vkq;
                }
            }
    }
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::sort(order.begin(), order.end(), [&](int x, int y) { return a[(size_t)x * n + x] < a[(size_t)y * n + y]; });
    std::vector<double> vs((size_t)n * n);
    w.resize(n);
    for (int k = 0; k < n; ++k) {
        w[k] = a[(size_t)order[k] * n + order[k]];
        for (int i = 0; i < n; ++i) vs[(size_t)i * n + k] = v[(size_t)i * n + order[k]];
    }
    v.swap(vs);
}

// Solve H y = b in place for a Hermitian positive-definite H (row-major), Cholesky.
bool hpd_solve(int n, const std::vector<cd> &h, std::vector<cd> &b) {
    std::vector<cd> l((size_t)n * n, cd(0.0, 0.0));
    for (int j = 0; j < n; ++j) {
        double d = h[(size_t)j * n + j].real();
        for (int k = 0; k < j; ++k) d -= std::norm(l[(size_t)j * n + k]);
        if (!(d > 0.0)) return false;
        const double ljj = std::sqrt(d);
        l[(size_t)j * n + j] = ljj;
        for (int i = j + 1; i < n; ++i) {
            cd sum = h[(size_t)i * n + j];
            for (int k = 0; k < j; ++k) sum -= l[(size_t)i * n + k] * std::conj(l[(size_t)j * n + k]);
            l[(size_t)i * n + j] = sum / ljj;
        }
    }
    for (int i = 0; i < n; ++i) {
        cd sum = b[i];
        for (int k = 0; k < i; ++k) sum -= l[(size_t)i * n + k] * b[k];
        b[i] = sum / l[(size_t)i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
        cd sum = b[i];
        for (int k = i + 1; k < n; ++k) sum -= std::conj(l[(size_t)k * n + i]) * b[k];
        b[i] = sum / l[(size_t)i * n + i];
    }
    return true;
}
}  // namespace

constexpr int EIG_RING = 128;  // >= the longest block of iterations between host reads

struct wl_eigcg {
    wl_ctx *c = nullptr;
    int op = WL_OP_DHAT, nev = 10, m = 60, max_vec = 0;
    double kappa = 0.0, mu = 0.0;
    int nh = 1;
    size_t fbytes = 0;   // one FP64 single-rhs field of the operator's subset
    long nelem = 0;      // complex doubles per field
    char *ubuf = nullptr, *aubuf = nullptr, *vbuf = nullptr, *wbuf = nullptr;
    double2 *coef = nullptr;
    double *hist = nullptr;  // ring of (alpha, beta) of the tracked CG run
    int *rec = nullptr;      // iterations recorded in the ring
    int nvec = 0;
    std::vector<cd> H;   // U^+ A U, row-major nvec x nvec
    std::vector<double> ritz;
    void *U(int k) const { return ubuf + (size_t)k * fbytes; }
    void *AU(int k) const { return aubuf + (size_t)k * fbytes; }
    void *V(int slot) const { return vbuf + (size_t)slot * fbytes; }
    void *W(int k) const { return wbuf + (size_t)k * fbytes; }  // r, p, q, t, tmp (odd)
};

extern "C" wl_status wl_eigcg_create(wl_ctx *c, wl_op op, double kappa, double mu, int nev, int m, int max_vectors,
                                     wl_eigcg **out) {
    g_err.clear();
    if (!c || !out) return fail(WL_ERR_ARG, "null argument");
    *out = nullptr;
    if (op != WL_OP_D && op != WL_OP_DHAT) return fail(WL_ERR_ARG, "bad operator %d", (int)op);
    if (!std::isfinite(kappa) || !std::isfinite(mu)) return fail(WL_ERR_ARG, "non-finite kappa or mu");
    if (nev < 1 || 2 * nev > LC_MAX_OUT || m < 2 * nev + 2 || m > LC_MAX_IN || max_vectors < 0)
        return fail(WL_ERR_ARG, "need 1 <= nev <= 16, 2 nev + 2 <= m <= 64, max_vectors >= 0");
    wl_eigcg *E = new wl_eigcg();
    E->c = c;
    E->op = op;
    E->kappa = kappa;
    E->mu = mu;
    E->nev = nev;
    E->m = m;
    E->max_vec = max_vectors;
    E->nh = op == WL_OP_D ? 2 : 1;
    E->fbytes = half_bytes(c, WL_F64, 1) * E->nh;
    E->nelem = (long)(E->fbytes / 16);
    hipError_t e = hipSuccess;
    if (max_vectors > 0) {
        e = hipMalloc(&E->ubuf, E->fbytes * max_vectors);
        if (e == hipSuccess) e = hipMalloc(&E->aubuf, E->fbytes * max_vectors);
    }
    if (e == hipSuccess) e = hipMalloc(&E->vbuf, E->fbytes * 2 * m);
    if (e == hipSuccess) e = hipMalloc(&E->wbuf, E->fbytes * 5);
    if (e == hipSuccess) e = hipMalloc(&E->coef, sizeof(double2) * LC_MAX_IN * LC_MAX_OUT);
    if (e == hipSuccess) e = hipMalloc(&E->hist, sizeof(double) * 2 * EIG_RING);
    if (e == hipSuccess) e = hipMalloc(&E->rec, 64);
    if (e != hipSuccess) {
        wl_eigcg_destroy(E);
        return fail(WL_ERR_NOMEM, "EigCG workspace: %s", hipGetErrorString(e));
    }
    const void *lk;
    size_t sl;
    wl_status st = get_links(c, WL_F64, 18, &lk, &sl);
    if (st) {
        wl_eigcg_destroy(E);
        return st;
    }
    *out = E;
    return WL_OK;
}

extern "C" wl_status wl_eigcg_destroy(wl_eigcg *E) {
    if (!E) return WL_OK;
    (void)hipDeviceSynchronize();
    for (void *p : {(void *)E->ubuf, (void *)E->aubuf, (void *)E->vbuf, (void *)E->wbuf, (void *)E->coef,
                    (void *)E->hist, (void *)E->rec})
        if (p) (void)hipFree(p);
    delete E;
    return WL_OK;
}

extern "C" wl_status wl_eigcg_vectors(const wl_eigcg *E, int *nvec, double *ritz) {
    g_err.clear();
    if (!E || !nvec) return fail(WL_ERR_ARG, "null argument");
    *nvec = E->nvec;
    if (ritz)
        for (int k = 0; k < E->nvec; ++k) ritz[k] = E->ritz[k];
    return WL_OK;
}

extern "C" wl_status wl_eigcg_eigenvalues(const wl_eigcg *E, int *n, double *vals) {
    g_err.clear();
    if (!E || !n) return fail(WL_ERR_ARG, "null argument");
    const int K = E->nvec;
    *n = K;
    if (!vals || K == 0) return WL_OK;
    // H = X + iY Hermitian: the real symmetric [[X, -Y], [Y, X]] has each eigenvalue of H twice
    const int n2 = 2 * K;
    std::vector<double> m((size_t)n2 * n2), w, v;
    for (int i = 0; i < K; ++i)
        for (int j = 0; j < K; ++j) {
            const cd h = 0.5 * (E->H[(size_t)i * K + j] + std::conj(E->H[(size_t)j * K + i]));
            m[(size_t)i * n2 + j] = m[(size_t)(i + K) * n2 + (j + K)] = h.real();
            m[(size_t)(i + K) * n2 + j] = h.imag();
            m[(size_t)i * n2 + (j + K)] = -h.imag();
        }
    sym_eig(n2, m, w, v);
    for (int k = 0; k < K; ++k) vals[k] = 0.5 * (w[2 * k] + w[2 * k + 1]);
    return WL_OK;
}

namespace {
// FP64 single-rhs field helpers of an EigCG context (all synchronous where they return a number)
struct EigOps {
    wl_eigcg *E;
    hipStream_t s;
    long stride;
    size_t hb;
    VecArgs vec(int n) const { return vec_args(E->c, WL_F64, 1); }
    wl_status apply_a(void *out, const void *in, double *pap) {
        // out = M^+ M in; *pap = ||M in||^2 (= <in, A in>) when pap != null
        wl_ctx *c = E->c;
        long nblk = 0;
        wl_status st = apply_m(c, E->op, false, E->kappa, WL_F64, 18, 1, E->W(3), in, E->W(4),
                               pap ? (double *)c->buf[S_PARTIALS] : nullptr, stride, nullptr, s, &nblk, E->mu);
        if (st) return st;
        if (pap && (st = reduce_to_host(c, 1, stride, nblk, pap, s))) return st;
        return apply_m(c, E->op, true, E->kappa, WL_F64, 18, 1, out, E->W(3), E->W(4), nullptr, 0, nullptr, s,
                       nullptr, E->mu);
    }
    wl_status dot(const void *x, const void *y, cd *out) {
        VecArgs v = vec_args(E->c, WL_F64, 1);
        set_vec(v, 0, x, hb);
        set_vec(v, 1, y, hb);
        v.partials = (double *)E->c->buf[S_PARTIALS];
        v.part_stride = stride;
        HIP_TRY(blas_dot(WL_F64, v, E->nh, s));
        double d[2];
        wl_status st = reduce_to_host(E->c, 2, stride, blas_blocks(v.n) * E->nh, d, s);
        *out = cd(d[0], d[1]);
        return st;
    }
    // y = a x + b y [, *n2 = ||y||^2]
    wl_status axpby(double a, const void *x, double b, void *y, double *n2) {
        VecArgs v = vec_args(E->c, WL_F64, 1);
        set_vec(v, 0, x, hb);
        set_vec(v, 1, y, hb);
        v.a = a;
        v.b = b;
        v.partials = (double *)E->c->buf[S_PARTIALS];
        v.part_stride = stride;
        HIP_TRY(blas_axpby(WL_F64, v, E->nh, n2 != nullptr, s));
        if (n2) return reduce_to_host(E->c, 1, stride, blas_blocks(v.n) * E->nh, n2, s);
        return WL_OK;
    }
    wl_status scale(double a, const void *x, void *y) {  // y = a x
        VecArgs v = vec_args(E->c, WL_F64, 1);
        set_vec(v, 0, x, hb);
        set_vec(v, 1, y, hb);
        v.a = a;
        v.b = 0.0;
        HIP_TRY(blas_twist(WL_F64, v, E->nh, s));
        return WL_OK;
    }
    // out[o] (+)= sum_j coef[j][o] in[j] for nin <= 64, nout <= 32 (coef row-major nin x nout)
    wl_status lincomb(const std::vector<const void *> &in, const std::vector<void *> &out, const std::vector<cd> &coef,
                      bool accumulate) {
        LinCombArgs a;
        std::memset(&a, 0, sizeof a);
        a.nin = (int)in.size();
        a.nout = (int)out.size();
        for (int j = 0; j < a.nin; ++j) a.in[j] = (const double2 *)in[j];
        for (int o = 0; o < a.nout; ++o) a.out[o] = (double2 *)out[o];
        std::vector<double2> h(coef.size());
        for (size_t k = 0; k < coef.size(); ++k) h[k] = make_double2(coef[k].real(), coef[k].imag());
        HIP_TRY(hipMemcpyAsync(E->coef, h.data(), sizeof(double2) * h.size(), hipMemcpyHostToDevice, s));
        a.coef = E->coef;
        a.accumulate = accumulate ? 1 : 0;
        a.n = E->nelem;
        HIP_TRY(blas_lincomb(a, s));
        HIP_TRY(hipStreamSynchronize(s));  // the coefficient buffer is reused by the next call
        return WL_OK;
    }
    // out[j * w.size() + o] = <in[j], w[o]> for any number of inputs (64 per launch), w.size() <= 16
    wl_status blockdot(const std::vector<const void *> &in, const std::vector<const void *> &w,
                       std::vector<cd> &out) {
        const int nw = (int)w.size();
        out.assign(in.size() * nw, cd(0.0, 0.0));
        if (in.empty() || nw == 0) return WL_OK;
        if (nw > BD_MAX_W) return fail(WL_ERR_ARG, "more than %d fields in a block inner product", BD_MAX_W);
        const long nb = blockdot_blocks(E->nelem);
        std::vector<double> d(2 * BD_MAX_IN * nw);
        double *dev = (double *)E->c->buf[S_SCAL];
        for (size_t j0 = 0; j0 < in.size(); j0 += BD_MAX_IN) {
            const int nj = (int)std::min<size_t>(BD_MAX_IN, in.size() - j0);
            BlockDotArgs a;
            std::memset(&a, 0, sizeof a);
            a.nin = nj;
            a.nw = nw;
            for (int k = 0; k < nj; ++k) a.in[k] = (const double2 *)in[j0 + k];
            for (int o = 0; o < nw; ++o) a.w[o] = (const double2 *)w[o];
            a.n = E->nelem;
            a.partials = (double *)E->c->buf[S_PARTIALS];
            a.stride = nb;
            HIP_TRY(blas_blockdot(a, s));
            HIP_TRY(reduce_rows(a.partials, nb, nb, 2 * nj * nw, dev, s));
            HIP_TRY(hipMemcpyAsync(d.data(), dev, sizeof(double) * 2 * nj * nw, hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            for (int k = 0; k < nj * nw; ++k) out[j0 * nw + k] = cd(d[2 * k], d[2 * k + 1]);
        }
        return WL_OK;
    }
    // outs[o] += sum_j c[j * outs.size() + o] in[j] for any number of inputs
    wl_status combine_into(const std::vector<const void *> &in, const std::vector<void *> &outs,
                           const std::vector<cd> &c) {
        const size_t no = outs.size();
        for (size_t j0 = 0; j0 < in.size(); j0 += LC_MAX_IN) {
            const size_t nj = std::min<size_t>(LC_MAX_IN, in.size() - j0);
            std::vector<const void *> part(in.begin() + j0, in.begin() + j0 + nj);
            std::vector<cd> cf(c.begin() + j0 * no, c.begin() + (j0 + nj) * no);
            wl_status st = lincomb(part, outs, cf, true);
            if (st) return st;
        }
        return WL_OK;
    }
    std::vector<const void *> space(int k) const {
        std::vector<const void *> u(k);
        for (int i = 0; i < k; ++i) u[i] = E->U(i);
        return u;
    }
};
}  // namespace

extern "C" wl_status wl_eigcg_solve(wl_eigcg *E, void *x, const void *b, double tol, int maxiter, int collect,
                                    wl_solver_info *info, void *stream) {
    g_err.clear();
    const auto t0 = std::chrono::steady_clock::now();
    if (!E) return fail(WL_ERR_ARG, "null EigCG context");
    wl_ctx *c = E->c;
    const int subset = E->op == WL_OP_D ? WL_FULL : WL_EVEN;
    wl_status st = check_field_args(c, subset, WL_F64, 1);
    if (st) return st;
    if (!x || !b || !aligned16(x) || !aligned16(b)) return fail(WL_ERR_ARG, "null or misaligned field pointer");
    if (!(tol > 0.0) || maxiter < 1) return fail(WL_ERR_ARG, "bad tolerance or iteration limit");
    if (overlap(x, E->fbytes, b, E->fbytes)) return fail(WL_ERR_ARG, "x and b overlap");
    EigOps O{E, (hipStream_t)stream, part_stride_for(c, 1), half_bytes(c, WL_F64, 1)};
    if ((st = ensure_buf(c, S_PARTIALS, sizeof(double) * std::max<long>(2 * O.stride, 2 * BD_MAX_IN * BD_MAX_W *
                                                                                          blockdot_blocks(E->nelem)))) ||
        (st = ensure_buf(c, S_SCAL, sizeof(double) * 2 * BD_MAX_IN * BD_MAX_W)))
        return st;
    void *r = E->W(0), *q = E->W(2);
    double b2 = 0.0;
    {
        cd d;
        if ((st = O.dot(b, b, &d))) return st;
        b2 = d.real();
    }
    wl_solver_info out{};
    // init-CG: x0 = U H^-1 U^+ b
    {
        VecArgs v = vec_args(c, WL_F64, 1);
        set_vec(v, 0, x, O.hb);
        HIP_TRY(blas_zero(WL_F64, v, E->nh, O.s));
    }
    if (E->nvec > 0 && b2 > 0.0) {
        const int K = E->nvec;
        const std::vector<const void *> us = O.space(K);
        std::vector<cd> y;
        if ((st = O.blockdot(us, {b}, y))) return st;
        if (!hpd_solve(K, E->H, y)) return fail(WL_BREAKDOWN, "deflation matrix not positive definite");
        if ((st = O.combine_into(us, {x}, y))) return st;
    }
    if (!(b2 > 0.0)) {
        HIP_TRY(hipStreamSynchronize(O.s));
        if (info) *info = out;
        return WL_OK;
    }
    const double target2 = tol * tol * b2;
    // search space (slots of vbuf), tridiagonal / projected matrix T, pending coupling after a restart
    // 2 m slots: the old basis, the restarted one and the next block of new vectors
    const int m = E->m, nev = E->nev, nslot = 2 * m;
    bool track = collect && E->nvec + nev <= E->max_vec;
    if (!track) {
        // nothing to collect: the library's CG from the init-CG guess
        wl_solver_params P;
        wl_solver_params_default(&P);
        P.tol = tol;
        P.maxiter = maxiter;
        P.mu = E->mu;
        wl_solver_info ci{};
        st = wl_cg_solve(c, x, b, (wl_op)E->op, E->kappa, 1, &P, &ci, stream);
        if (st < 0) return st;
        HIP_TRY(hipStreamSynchronize(O.s));
        ci.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        if (info) *info = ci;
        return st;
    }
    // One tracked CG run on device scalars (the Lanczos relation holds within one
    // uninterrupted run).  Before each iteration a kernel stores r / ||r|| in the next
    // free slot of the search space; after it another appends the iteration's alpha
    // and beta to a ring.  The host reads both only when the space is full (restart)
    // or every check_every iterations, and builds T from them.
    wl_solver_params P;
    wl_solver_params_default(&P);
    P.tol = tol;
    P.maxiter = maxiter;
    P.mu = E->mu;
    CGRun R;
    if ((st = cg_setup(c, x, b, E->op, E->kappa, 1, P, O.s, R))) return st;
    // pinned host copies: the scalars at offset 0, the (alpha, beta) ring at 256 (so the
    // reads are truly asynchronous and the host work of a restart overlaps the device)
    static_assert(sizeof(CGScalars) <= 256, "CGScalars larger than its pinned slot");
    if ((st = ensure_pinned(c, 256 + sizeof(double) * 2 * EIG_RING))) return st;
    const double *hh = (const double *)((const char *)c->host_pinned + 256);
    {
        VecArgs v = vec_args(c, WL_F64, 1);
        set_vec(v, 0, b, R.hb_hi);
        v.partials = R.partials;
        v.part_stride = R.stride;
        HIP_TRY(blas_norm2(WL_F64, v, R.nh, R.s));
        HIP_TRY(reduce_partials(R.partials, R.stride, R.nblk_blas, 1, R.bnorm2, R.s));
    }
    if ((st = true_residual(R))) return st;
    HIP_TRY(cg_init(R.sc, 1, R.partials, R.stride, R.nblk_blas, R.bnorm2, tol, maxiter, R.done, R.s));
    if ((st = load_residual(R))) return st;
    HIP_TRY(hipMemsetAsync(E->rec, 0, sizeof(int), R.s));
    std::vector<int> cols;  // physical slot of each column
    std::vector<char> used(nslot, 0);
    std::vector<double> T((size_t)m * m, 0.0), pending;
    auto take_slot = [&](int *slot) -> bool {
        int sl = 0;
        while (sl < nslot && used[sl]) ++sl;
        if (sl == nslot) return false;
        used[sl] = 1;
        *slot = sl;
        return true;
    };
    // A restart (the space is full) is scheduled at a host read and carried out after
    // the next block of iterations has been enqueued, so that its host part (two small
    // eigenproblems) overlaps the device work; the recombination of the old basis is
    // enqueued behind that block, into slots reserved for it.
    struct Restart {
        bool due = false;
        std::vector<double> T;      // T_m of the full space
        std::vector<int> old_cols;  // its basis
        std::vector<int> reserved;  // slots of the restarted basis (the first columns now)
        double off = 0.0;           // coupling of the m-th column to the next vector
    } rs;
    auto do_restart = [&]() -> wl_status {
        // the nev lowest Ritz vectors of T_m and of T_{m-1}
        const std::vector<double> &To = rs.T;
        std::vector<double> tm((size_t)m * m), tm1((size_t)(m - 1) * (m - 1)), w, Y, w1, Y1;
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) tm[(size_t)i * m + j] = To[(size_t)i * m + j];
        for (int i = 0; i < m - 1; ++i)
            for (int j = 0; j < m - 1; ++j) tm1[(size_t)i * (m - 1) + j] = To[(size_t)i * m + j];
        sym_eig(m, tm, w, Y);
        sym_eig(m - 1, tm1, w1, Y1);
        // Z = [Y(:, :nev), [Y1(:, :nev); 0]], orthonormalised (two Gram-Schmidt passes)
        std::vector<std::vector<double>> Z;
        for (int j = 0; j < 2 * nev; ++j) {
            std::vector<double> z(m, 0.0);
            for (int i = 0; i < m; ++i)
                z[i] = j < nev ? Y[(size_t)i * m + j] : (i < m - 1 ? Y1[(size_t)i * (m - 1) + (j - nev)] : 0.0);
            for (int pass = 0; pass < 2; ++pass)
                for (auto &zz : Z) {
                    double d = 0.0;
                    for (int i = 0; i < m; ++i) d += zz[i] * z[i];
                    for (int i = 0; i < m; ++i) z[i] -= d * zz[i];
                }
            double nz = 0.0;
            for (int i = 0; i < m; ++i) nz += z[i] * z[i];
            nz = std::sqrt(nz);
            if (nz < 1e-10) continue;
            for (int i = 0; i < m; ++i) z[i] /= nz;
            Z.push_back(z);
        }
        const int kq = (int)Z.size(), nres = (int)rs.reserved.size();
        std::vector<const void *> in(m);
        for (int i = 0; i < m; ++i) in[i] = E->V(rs.old_cols[i]);
        std::vector<void *> outs(kq);
        for (int j = 0; j < kq; ++j) outs[j] = E->V(rs.reserved[j]);
        std::vector<cd> cf((size_t)m * kq);
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < kq; ++j) cf[(size_t)i * kq + j] = Z[j][i];
        wl_status e2 = O.lincomb(in, outs, cf, false);
        if (e2) return e2;
        for (int sl : rs.old_cols) used[sl] = 0;
        // reserved slots the restarted basis does not need
        for (int j = kq; j < nres; ++j) used[rs.reserved[j]] = 0;
        cols.erase(cols.begin() + kq, cols.begin() + nres);
        // T <- Z^T T_m Z, and the next vector couples through the last row of Z
        std::fill(T.begin(), T.end(), 0.0);
        for (int a = 0; a < kq; ++a)
            for (int bb = 0; bb < kq; ++bb) {
                double sum = 0.0;
                for (int i = 0; i < m; ++i)
                    for (int j = 0; j < m; ++j) sum += Z[a][i] * To[(size_t)i * m + j] * Z[bb][j];
                T[(size_t)a * m + bb] = sum;
            }
        pending.assign(kq, 0.0);
        for (int a = 0; a < kq; ++a) pending[a] = Z[a][m - 1] * rs.off;
        rs.due = false;
        return WL_OK;
    };
    CGScalars hs{};
    int seen = 0;  // iterations whose step lengths are in T
    double alpha_old = 0.0, beta_old = 0.0;
    bool have_old = false;
    for (;;) {
        const int block = std::max(1, std::min(P.check_every, m - (int)cols.size()));
        size_t ncols0 = cols.size();
        for (int j = 0; j < block; ++j) {
            int slot = 0;
            if (!take_slot(&slot)) return fail(WL_ERR_ARG, "EigCG search space has no free slot (internal)");
            cols.push_back(slot);
            VecArgs v = vec_args(c, WL_F64, 1);
            set_vec(v, 0, R.r, R.hb_hi);
            set_vec(v, 1, E->V(slot), R.hb_hi);
            v.sc = R.sc;
            v.flag = R.done;
            HIP_TRY(blas_scale_by_rho(v, R.nh, R.s));
            if ((st = cg_iteration(R, false))) return st;
            HIP_TRY(cg_record(R.sc, E->hist, EIG_RING, E->rec, R.s));
        }
        HIP_TRY(hipMemcpyAsync(c->host_pinned, R.sc, sizeof(CGScalars), hipMemcpyDeviceToHost, R.s));
        HIP_TRY(hipMemcpyAsync((char *)c->host_pinned + 256, E->hist, sizeof(double) * 2 * EIG_RING,
                               hipMemcpyDeviceToHost, R.s));
        if (rs.due) {
            const size_t before = cols.size();
            if ((st = do_restart())) return st;
            ncols0 -= before - cols.size();
        }
        HIP_TRY(hipStreamSynchronize(R.s));
        std::memcpy(&hs, c->host_pinned, sizeof hs);
        if (hs.status == WL_BREAKDOWN) return fail(WL_BREAKDOWN, "EigCG breakdown: <p, A p> <= 0 or not finite");
        // slots issued for iterations that did not run (the run stopped) were never written
        const int nnew = hs.iter - seen;
        const size_t keep = ncols0 + (size_t)nnew;
        for (size_t i = keep; i < cols.size(); ++i) used[cols[i]] = 0;
        cols.resize(keep);
        for (int t = 0; t < nnew; ++t) {
            const int g = seen + t, k = (int)ncols0 + t + 1;
            const double alpha = hh[2 * (g % EIG_RING)], beta = hh[2 * (g % EIG_RING) + 1];
            T[(size_t)(k - 1) * m + (k - 1)] = 1.0 / alpha + (have_old ? beta_old / alpha_old : 0.0);
            if (!pending.empty()) {
                for (int i2 = 0; i2 < k - 1; ++i2) T[(size_t)i2 * m + (k - 1)] = T[(size_t)(k - 1) * m + i2] = pending[i2];
                pending.clear();
            }
            const double off = -std::sqrt(beta) / alpha;
            if (k == m) {
                // full: schedule the restart (only the last new column can fill the space)
                rs.due = true;
                rs.T = T;
                rs.old_cols = cols;
                rs.off = off;
                rs.reserved.clear();
                for (int j = 0; j < 2 * nev; ++j) {
                    int slot = 0;
                    if (!take_slot(&slot)) return fail(WL_ERR_ARG, "EigCG search space has no free slot (internal)");
                    rs.reserved.push_back(slot);
                }
                cols = rs.reserved;
            } else {
                T[(size_t)(k - 1) * m + k] = T[(size_t)k * m + (k - 1)] = off;
            }
            alpha_old = alpha;
            beta_old = beta;
            have_old = true;
        }
        seen = hs.iter;
        if (!hs.active) break;
    }
    if (rs.due && (st = do_restart())) return st;
    int total = hs.iter, restarts = 0;
    double rho = hs.rho, true2 = 0.0;
    // FP64 true residual; if it misses the tolerance, finish untracked with the library's CG
    if ((st = O.apply_a(q, x, nullptr)) || (st = O.scale(1.0, b, r)) || (st = O.axpby(-1.0, q, 1.0, r, &true2)))
        return st;
    if (true2 > target2 && total < maxiter) {
        P.maxiter = maxiter - total;
        wl_solver_info ci{};
        st = wl_cg_solve(c, x, b, (wl_op)E->op, E->kappa, 1, &P, &ci, stream);
        if (st < 0) return st;
        total += ci.iters;
        restarts += 1 + ci.restarts;
        rho = ci.rel_resid * ci.rel_resid * b2;
        true2 = ci.true_rel_resid * ci.true_rel_resid * b2;
    }
    // keep the nev lowest Ritz vectors of the tracked space
    if (collect && track && !cols.empty()) {
        const int k = (int)cols.size();
        std::vector<double> tk((size_t)k * k), w, Y;
        for (int i = 0; i < k; ++i)
            for (int j = 0; j < k; ++j) tk[(size_t)i * k + j] = T[(size_t)i * m + j];
        sym_eig(k, tk, w, Y);
        const int nr = std::min(nev, k);
        std::vector<const void *> in(k);
        for (int i = 0; i < k; ++i) in[i] = E->V(cols[i]);
        std::vector<int> fresh;
        for (int sl = 0; sl < nslot && (int)fresh.size() < nr; ++sl)
            if (!used[sl]) fresh.push_back(sl);
        std::vector<void *> outs(nr);
        for (int j = 0; j < nr; ++j) outs[j] = E->V(fresh[j]);
        std::vector<cd> cf((size_t)k * nr);
        for (int i = 0; i < k; ++i)
            for (int j = 0; j < nr; ++j) cf[(size_t)i * nr + j] = Y[(size_t)i * k + j];
        if ((st = O.lincomb(in, outs, cf, false))) return st;
        // classical Gram-Schmidt of the block against U, twice (one pass over U per step)
        const int K0 = E->nvec;
        const std::vector<const void *> us = O.space(K0), wc(outs.begin(), outs.end());
        for (int pass = 0; pass < 2 && K0 > 0; ++pass) {
            std::vector<cd> C;
            if ((st = O.blockdot(us, wc, C))) return st;
            for (auto &z : C) z = -z;
            if ((st = O.combine_into(us, outs, C))) return st;
        }
        // then each vector against those already kept from this block, normalised, A applied
        std::vector<double> rqs;
        for (int j = 0; j < nr && E->nvec < E->max_vec; ++j) {
            void *wv = outs[j];
            const int K = E->nvec;
            std::vector<const void *> kept;
            for (int i = K0; i < K; ++i) kept.push_back(E->U(i));
            for (int pass = 0; pass < 2 && !kept.empty(); ++pass) {
                std::vector<cd> d;
                if ((st = O.blockdot(kept, {wv}, d))) return st;
                for (auto &z : d) z = -z;
                if ((st = O.combine_into(kept, {wv}, d))) return st;
            }
            cd n2;
            if ((st = O.dot(wv, wv, &n2))) return st;
            if (!(n2.real() > 1e-20)) continue;
            if ((st = O.scale(1.0 / std::sqrt(n2.real()), wv, E->U(K)))) return st;
            double rq = 0.0;
            if ((st = O.apply_a(E->AU(K), E->U(K), &rq))) return st;
            rqs.push_back(rq);
            E->nvec = K + 1;
        }
        // the new columns of H = U^+ A U in one pass over U
        const int K1 = E->nvec, nn = K1 - K0;
        if (nn > 0) {
            std::vector<const void *> anew;
            for (int i = K0; i < K1; ++i) anew.push_back(E->AU(i));
            std::vector<cd> C;
            if ((st = O.blockdot(O.space(K1), anew, C))) return st;
            std::vector<cd> Hn((size_t)K1 * K1);
            for (int i = 0; i < K0; ++i)
                for (int jj = 0; jj < K0; ++jj) Hn[(size_t)i * K1 + jj] = E->H[(size_t)i * K0 + jj];
            for (int jn = 0; jn < nn; ++jn) {
                const int jj = K0 + jn;
                for (int i = 0; i < jj; ++i) {
                    Hn[(size_t)i * K1 + jj] = C[(size_t)i * nn + jn];
                    Hn[(size_t)jj * K1 + i] = std::conj(C[(size_t)i * nn + jn]);
                }
                Hn[(size_t)jj * K1 + jj] = cd(rqs[jn], 0.0);
                E->ritz.push_back(rqs[jn]);
            }
            E->H.swap(Hn);
        }
    }
    HIP_TRY(hipStreamSynchronize(O.s));
    out.iters = total;
    out.restarts = restarts;
    out.rel_resid = std::sqrt(rho / b2);
    out.true_rel_resid = std::sqrt(true2 / b2);
    out.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (info) *info = out;
    if (true2 > target2) return fail(WL_NOT_CONVERGED, "EigCG did not reach the tolerance");
    return WL_OK;
}

// ------------------------------------------------------------------ link-spinor access kernel
extern "C" wl_status wl_su3_apply(void *psi, const void *u, const void *phi, long n, int mode, int layout,
                                  const int *index, const unsigned long long *ptrs, void *stream) {
    g_err.clear();
    if (n < 0) return fail(WL_ERR_ARG, "n = %ld < 0", n);
    if (mode < WL_ACCESS_SEQ || mode > WL_ACCESS_PTR) return fail(WL_ERR_ARG, "bad access mode %d", mode);
    if (layout < 0 || layout > 1) return fail(WL_ERR_ARG, "bad layout %d", layout);
    if (n == 0) return WL_OK;
    if (mode != WL_ACCESS_PTR && (!psi || !u || !phi || !aligned16(psi) || !aligned16(u) || !aligned16(phi)))
        return fail(WL_ERR_ARG, "null or misaligned field pointer");
    if (mode == WL_ACCESS_INDEX && !index) return fail(WL_ERR_ARG, "index mode without an index array");
    if (mode == WL_ACCESS_PTR && !ptrs) return fail(WL_ERR_ARG, "pointer mode without an address array");
    if (n > (long)INT32_MAX) return fail(WL_ERR_ARG, "n = %ld too large", n);
    AccessArgs a{(double2 *)psi, (const double2 *)u, (const double2 *)phi, n, index, ptrs};
    HIP_TRY(launch_su3_apply(a, mode, layout, (hipStream_t)stream));
    return WL_OK;
}

// ------------------------------------------------------------------ timing API
extern "C" wl_status wl_timing_enable(wl_ctx *c, int enable) {
    g_err.clear();
    if (!c) return fail(WL_ERR_ARG, "null context");
    if (enable < 0) return fail(WL_ERR_ARG, "enable = %d < 0", enable);
    HIP_TRY(hipDeviceSynchronize());
    c->timed.clear();
    c->pool_used = 0;
    c->timing = enable != 0;
    c->timing_stride = enable > 0 ? enable : 1;
    c->timing_seq = 0;
    return WL_OK;
}

extern "C" wl_status wl_timing_read(wl_ctx *c, wl_prec prec, int recon, int dagger, int epilogue, int *count,
                                    double *total_ms) {
    g_err.clear();
    if (!c || !count || !total_ms) return fail(WL_ERR_ARG, "null argument");
    if (!prec_ok(prec) || !recon_ok(prec, recon) || epilogue < 0 || epilogue > 7)
        return fail(WL_ERR_ARG, "bad kernel selector");
    const int key = timing_key(prec, recon, dagger != 0, epilogue);
    int n = 0;
    double ms = 0.0;
    for (auto &t : c->timed) {
        if (t.key != key) continue;
        HIP_TRY(hipEventSynchronize(t.ev[1]));
        float m = 0.f;
        HIP_TRY(hipEventElapsedTime(&m, t.ev[0], t.ev[1]));
        ms += m;
        ++n;
    }
    *count = n;
    *total_ms = ms;
    return WL_OK;
}

// ------------------------------------------------------------------ launch configuration
extern "C" wl_status wl_ctx_set_launch(wl_ctx *c, wl_prec prec, const wl_launch *l) {
    g_err.clear();
    if (!c || !l) return fail(WL_ERR_ARG, "null argument");
    if (!prec_ok(prec)) return fail(WL_ERR_ARG, "bad precision %d", (int)prec);
    if (const char *why = launch_problem(l->block, l->tps, l->nt, l->rpt))
        return fail(WL_ERR_ARG, "launch (block %d, tps %d, nt %d, rpt %d): %s", l->block, l->tps, l->nt, l->rpt, why);
    LaunchCfg &g = c->cfg[prec];
    g.block = l->block;
    g.swizzle = l->swizzle ? 1 : 0;
    g.tps = l->tps;
    g.tchunk = l->tchunk;
    g.nt = l->nt;
    g.rpt = l->rpt;
    return WL_OK;
}

extern "C" wl_status wl_ctx_get_launch(const wl_ctx *c, wl_prec prec, wl_launch *l) {
    g_err.clear();
    if (!c || !l) return fail(WL_ERR_ARG, "null argument");
    if (!prec_ok(prec)) return fail(WL_ERR_ARG, "bad precision %d", (int)prec);
    const LaunchCfg &g = c->cfg[prec];
    l->block = g.block;
    l->swizzle = g.swizzle;
    l->tps = g.tps;
    l->tchunk = g.tchunk;
    l->nt = g.nt;
    l->rpt = g.rpt;
    return WL_OK;
}

// ------------------------------------------------------------------ PTC preconditioner
struct wl_ptc {
    int channels;
    long n1, n2;          // complex weights of layer 1 (9 x C x 1 x 16) and layer 2 (9 x 1 x C x 16)
    float *w = nullptr;   // FP32 master weights, layer 1 then layer 2, (re, im) interleaved
    uint16_t *wb = nullptr;  // BF16 copy used by the kernels
    double *grad = nullptr;  // dL/dW* accumulated, complex (re, im)
    float *m = nullptr, *v = nullptr;  // Adam moments per real parameter
    double *loss = nullptr;  // accumulated loss (device)
    int t = 0;               // Adam steps taken
};

extern "C" wl_status wl_ptc_create(int channels, const double *w1, const double *w2, wl_ptc **out) {
    g_err.clear();
    if (!w1 || !w2 || !out) return fail(WL_ERR_ARG, "null argument");
    *out = nullptr;
    if (channels < 1 || channels > PTC_MAXC) return fail(WL_ERR_ARG, "channels %d not in [1, %d]", channels, PTC_MAXC);
    wl_ptc *n = new wl_ptc();
    n->channels = channels;
    n->n1 = (long)PTC_NPATH * channels * 16;
    n->n2 = n->n1;
    const long nr = 2 * (n->n1 + n->n2);  // real parameters
    std::vector<float> host(nr);
    for (long k = 0; k < 2 * n->n1; ++k) host[k] = (float)w1[k];
    for (long k = 0; k < 2 * n->n2; ++k) host[2 * n->n1 + k] = (float)w2[k];
    hipError_t e = hipSuccess;
    if ((e = hipMalloc(&n->w, nr * sizeof(float))) != hipSuccess || (e = hipMalloc(&n->wb, nr * sizeof(uint16_t))) != hipSuccess ||
        (e = hipMalloc(&n->grad, nr * sizeof(double))) != hipSuccess || (e = hipMalloc(&n->m, nr * sizeof(float))) != hipSuccess ||
        (e = hipMalloc(&n->v, nr * sizeof(float))) != hipSuccess || (e = hipMalloc(&n->loss, sizeof(double))) != hipSuccess) {
        (void)hipGetLastError();
        wl_ptc_destroy(n);
        return fail(WL_ERR_NOMEM, "hipMalloc of PTC weights failed: %s", hipGetErrorString(e));
    }
    if ((e = hipMemcpy(n->w, host.data(), nr * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemset(n->grad, 0, nr * sizeof(double))) != hipSuccess ||
        (e = hipMemset(n->m, 0, nr * sizeof(float))) != hipSuccess ||
        (e = hipMemset(n->v, 0, nr * sizeof(float))) != hipSuccess ||
        (e = hipMemset(n->loss, 0, sizeof(double))) != hipSuccess || (e = launch_to_bf16(n->w, n->wb, nr, 0)) != hipSuccess ||
        (e = hipDeviceSynchronize()) != hipSuccess) {
        wl_ptc_destroy(n);
        return fail(WL_ERR_HIP, "PTC weight initialisation failed: %s", hipGetErrorString(e));
    }
    *out = n;
    return WL_OK;
}

extern "C" wl_status wl_ptc_destroy(wl_ptc *n) {
    if (!n) return WL_OK;
    (void)hipDeviceSynchronize();
    if (n->w) (void)hipFree(n->w);
    if (n->wb) (void)hipFree(n->wb);
    if (n->grad) (void)hipFree(n->grad);
    if (n->m) (void)hipFree(n->m);
    if (n->v) (void)hipFree(n->v);
    if (n->loss) (void)hipFree(n->loss);
    delete n;
    return WL_OK;
}

static wl_status ptc_download(const wl_ptc *n, const void *src, bool is_double, double *w1, double *w2) {
    const long nr = 2 * (n->n1 + n->n2);
    std::vector<double> h(nr);
    if (is_double) {
        HIP_TRY(hipMemcpy(h.data(), src, nr * sizeof(double), hipMemcpyDeviceToHost));
    } else {
        std::vector<float> f(nr);
        HIP_TRY(hipMemcpy(f.data(), src, nr * sizeof(float), hipMemcpyDeviceToHost));
        for (long k = 0; k < nr; ++k) h[k] = f[k];
    }
    if (w1) std::memcpy(w1, h.data(), 2 * n->n1 * sizeof(double));
    if (w2) std::memcpy(w2, h.data() + 2 * n->n1, 2 * n->n2 * sizeof(double));
    return WL_OK;
}

extern "C" wl_status wl_ptc_get_weights(const wl_ptc *n, double *w1, double *w2) {
    g_err.clear();
    if (!n) return fail(WL_ERR_ARG, "null network");
    HIP_TRY(hipDeviceSynchronize());
    return ptc_download(n, n->w, false, w1, w2);
}

extern "C" wl_status wl_ptc_get_grads(const wl_ptc *n, double *g1, double *g2) {
    g_err.clear();
    if (!n) return fail(WL_ERR_ARG, "null network");
    HIP_TRY(hipDeviceSynchronize());
    return ptc_download(n, n->grad, true, g1, g2);
}

// bytes of a C-channel PTC field: C consecutive FULL FP32 single-rhs fields
static size_t ptc_field_bytes(const wl_ctx *c, int channels) {
    return (size_t)channels * 2 * half_bytes(c, WL_F32, 1);
}

static PtcArgs ptc_args(wl_ctx *c, void *out, const void *in, int cout, int cin, const void *w, int adjoint,
                        wl_status *st) {
    PtcArgs a;
    std::memset(&a, 0, sizeof a);
    const void *gauge = nullptr;
    size_t slab = 0;
    *st = get_links(c, WL_F32, 18, &gauge, &slab);
    a.g = c->g;
    (void)cin;
    a.out = (char *)out;
    a.in = (const char *)in;
    a.half = half_bytes(c, WL_F32, 1);
    a.gauge = gauge;
    a.slab_bytes = slab;
    a.w = w;
    a.cout = cout;
    a.cin = cin;
    a.adjoint = adjoint;
    a.vh = c->Vh;
    return a;
}

// out = M(in) = layer2(layer1(in)) with the BF16 weights; the hidden field is
// returned in `hidden` (channels C)
static wl_status ptc_forward(wl_ctx *c, const wl_ptc *n, void *out, const void *in, void *hidden, hipStream_t s) {
    wl_status st;
    PtcArgs a1 = ptc_args(c, hidden, in, n->channels, 1, n->wb, 0, &st);
    if (st) return st;
    HIP_TRY(launch_ptc_layer(a1, true, s));
    PtcArgs a2 = ptc_args(c, out, hidden, 1, n->channels, n->wb + 2 * n->n1, 0, &st);
    if (st) return st;
    HIP_TRY(launch_ptc_layer(a2, true, s));
    return WL_OK;
}

extern "C" wl_status wl_ptc_apply(wl_ctx *c, const wl_ptc *n, void *out, const void *in, void *stream) {
    g_err.clear();
    if (!c || !n || !out || !in || !aligned16(out) || !aligned16(in)) return fail(WL_ERR_ARG, "null or misaligned argument");
    const size_t hb = half_bytes(c, WL_F32, 1);
    if (overlap(out, 2 * hb, in, 2 * hb)) return fail(WL_ERR_ARG, "out and in overlap");
    wl_status st = ensure_buf(c, S_PTC_H, ptc_field_bytes(c, n->channels));
    if (st) return st;
    return ptc_forward(c, n, out, in, c->buf[S_PTC_H], (hipStream_t)stream);
}

extern "C" wl_status wl_ptc_layer(wl_ctx *c, void *out, const void *in, const float *weights, int cout, int cin,
                                  int adjoint, void *stream) {
    g_err.clear();
    if (!c || !out || !in || !weights || !aligned16(out) || !aligned16(in)) return fail(WL_ERR_ARG, "null or misaligned argument");
    if (cout < 1 || cin < 1 || cout * cin > PTC_MAXC) return fail(WL_ERR_ARG, "channels %d x %d exceed %d", cout, cin, PTC_MAXC);
    if (overlap(out, ptc_field_bytes(c, cout), in, ptc_field_bytes(c, cin)))
        return fail(WL_ERR_ARG, "out and in overlap");
    wl_status st;
    PtcArgs a = ptc_args(c, out, in, cout, cin, weights, adjoint ? 1 : 0, &st);
    if (st) return st;
    HIP_TRY(launch_ptc_layer(a, false, (hipStream_t)stream));
    return WL_OK;
}

extern "C" wl_status wl_ptc_weight_grad(wl_ctx *c, double *grad, const void *gout, const void *in, int cout, int cin,
                                        int accumulate, void *stream) {
    g_err.clear();
    if (!c || !grad || !gout || !in) return fail(WL_ERR_ARG, "null argument");
    if (cout < 1 || cin < 1 || cout * cin > PTC_MAXC) return fail(WL_ERR_ARG, "bad channel counts");
    const int ncombo = PTC_NPATH * cout * cin;
    const int nchunks = std::max(1, std::min(64, (int)(2048 / ncombo)));
    wl_status st = ensure_buf(c, S_PTC_PART, sizeof(float) * 32 * (size_t)ncombo * nchunks);
    if (st) return st;
    const void *gauge;
    size_t slab;
    if ((st = get_links(c, WL_F32, 18, &gauge, &slab))) return st;
    PtcGradArgs a;
    std::memset(&a, 0, sizeof a);
    a.g = c->g;
    a.gout = (const char *)gout;
    a.in = (const char *)in;
    a.half = half_bytes(c, WL_F32, 1);
    a.gauge = gauge;
    a.slab_bytes = slab;
    a.cout = cout;
    a.cin = cin;
    a.vh = c->Vh;
    a.partials = (float *)c->buf[S_PTC_PART];
    a.nchunks = nchunks;
    HIP_TRY(launch_ptc_wgrad(a, grad, accumulate, (hipStream_t)stream));
    return WL_OK;
}

// back-propagation of go = dL/d conj(M(r)) through both layers into the gradient accumulators
static wl_status ptc_backward(wl_ctx *c, wl_ptc *n, const void *go, const void *r, const void *h, void *gh,
                              void *stream) {
    const int C = n->channels;
    double *g1 = n->grad, *g2 = n->grad + 2 * n->n1;
    wl_status st;
    if ((st = wl_ptc_weight_grad(c, g2, go, h, 1, C, 1, stream))) return st;
    PtcArgs a2t = ptc_args(c, gh, go, C, 1, n->wb + 2 * n->n1, 1, &st);
    if (st) return st;
    HIP_TRY(launch_ptc_layer(a2t, true, (hipStream_t)stream));
    return wl_ptc_weight_grad(c, g1, gh, r, C, 1, 1, stream);
}

// ||f||^2 of one FULL FP32 field into the device scalar *dst
static hipError_t full_norm2_f32(wl_ctx *c, const void *f, double *dst, hipStream_t s) {
    const long stride = part_stride_for(c, 1);
    double *partials = (double *)c->buf[S_PARTIALS];
    VecArgs v = vec_args(c, WL_F32, 1);
    set_vec(v, 0, f, half_bytes(c, WL_F32, 1));
    v.partials = partials;
    v.part_stride = stride;
    hipError_t e = blas_norm2(WL_F32, v, 2, s);
    if (e != hipSuccess) return e;
    return reduce_partials(partials, stride, blas_blocks(v.n) * 2, 1, dst, s);
}

static wl_status ptc_workspace(wl_ctx *c, int C) {
    const size_t h1 = half_bytes(c, WL_F32, 1), fc = ptc_field_bytes(c, C);
    wl_status st;
    if ((st = ensure_buf(c, S_PTC_H, fc)) || (st = ensure_buf(c, S_PTC_GH, fc)) ||
        (st = ensure_buf(c, S_PTC_O, 2 * h1)) || (st = ensure_buf(c, S_PTC_GO, 2 * h1)) ||
        (st = ensure_buf(c, S_PTC_E2, sizeof(double) * 2)) ||
        (st = ensure_buf(c, S_PARTIALS, sizeof(double) * 2 * part_stride_for(c, 1))))
        return st;
    return WL_OK;
}

extern "C" wl_status wl_ptc_accumulate(wl_ctx *c, wl_ptc *n, const void *r, const void *e, double inv_npairs,
                                       void *stream) {
    g_err.clear();
    if (!c || !n || !r || !e || !aligned16(r) || !aligned16(e)) return fail(WL_ERR_ARG, "null or misaligned argument");
    if (!(inv_npairs > 0.0) || !std::isfinite(inv_npairs)) return fail(WL_ERR_ARG, "bad pair weight");
    hipStream_t s = (hipStream_t)stream;
    wl_status st;
    if ((st = ptc_workspace(c, n->channels))) return st;
    void *h = c->buf[S_PTC_H], *gh = c->buf[S_PTC_GH], *o = c->buf[S_PTC_O], *go = c->buf[S_PTC_GO];
    double *e2 = (double *)c->buf[S_PTC_E2];
    if ((st = ptc_forward(c, n, o, r, h, s))) return st;
    HIP_TRY(full_norm2_f32(c, e, e2, s));
    // loss and dL/d conj(out) = (out - e) / (N ||e||^2)
    HIP_TRY(launch_ptc_loss(o, e, go, c->Vh, e2, inv_npairs, (double *)c->buf[S_PARTIALS], part_stride_for(c, 1),
                            n->loss, s));
    return ptc_backward(c, n, go, r, h, gh, stream);
}

extern "C" wl_status wl_ptc_accumulate_residual(wl_ctx *c, wl_ptc *n, const void *r, double kappa,
                                                double inv_npairs, void *stream) {
    g_err.clear();
    if (!c || !n || !r || !aligned16(r)) return fail(WL_ERR_ARG, "null or misaligned argument");
    if (!(inv_npairs > 0.0) || !std::isfinite(inv_npairs)) return fail(WL_ERR_ARG, "bad pair weight");
    if (!std::isfinite(kappa)) return fail(WL_ERR_ARG, "non-finite kappa");
    hipStream_t s = (hipStream_t)stream;
    wl_status st;
    if ((st = ptc_workspace(c, n->channels))) return st;
    void *h = c->buf[S_PTC_H], *gh = c->buf[S_PTC_GH], *o = c->buf[S_PTC_O], *go = c->buf[S_PTC_GO];
    double *r2 = (double *)c->buf[S_PTC_E2];
    if ((st = ptc_forward(c, n, o, r, h, s))) return st;
    // y = D M(r) in go; then, in place, y <- (y - r) / (N ||r||^2) with the loss summed on the way
    if ((st = apply_m(c, WL_OP_D, false, kappa, WL_F32, 18, 1, go, o, nullptr, nullptr, 0, nullptr, s, nullptr)))
        return st;
    HIP_TRY(full_norm2_f32(c, r, r2, s));
    HIP_TRY(launch_ptc_loss(go, r, go, c->Vh, r2, inv_npairs, (double *)c->buf[S_PARTIALS], part_stride_for(c, 1),
                            n->loss, s));
    // dL/d conj(M(r)) = D^+ of that, written over the network output (no longer needed)
    if ((st = apply_m(c, WL_OP_D, true, kappa, WL_F32, 18, 1, o, go, nullptr, nullptr, 0, nullptr, s, nullptr)))
        return st;
    return ptc_backward(c, n, o, r, h, gh, stream);
}

extern "C" wl_status wl_ptc_step(wl_ptc *n, double lr, double *loss, void *stream) {
    g_err.clear();
    if (!n) return fail(WL_ERR_ARG, "null network");
    if (!(lr > 0.0) || !std::isfinite(lr)) return fail(WL_ERR_ARG, "bad learning rate");
    hipStream_t s = (hipStream_t)stream;
    n->t += 1;
    HIP_TRY(launch_adam(n->w, n->wb, n->grad, n->m, n->v, 2 * (n->n1 + n->n2), lr, 0.9, 0.999, 1e-8, n->t, s));
    double l = 0.0;
    HIP_TRY(hipMemcpyAsync(&l, n->loss, sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemsetAsync(n->loss, 0, sizeof(double), s));
    HIP_TRY(hipStreamSynchronize(s));
    if (loss) *loss = l;
    return WL_OK;
}

// ------------------------------------------------------------------ FGCR and CGNR
namespace {
// host-side scalar helpers for the FGCR driver (FULL fields, one rhs)
struct Fields {
    wl_ctx *c;
    hipStream_t s;
    long stride;
};
}  // namespace

static wl_status dot_full(Fields &F, int prec, const void *x, const void *y, double out[2]) {
    wl_ctx *c = F.c;
    VecArgs v = vec_args(c, prec, 1);
    const size_t hb = half_bytes(c, prec, 1);
    set_vec(v, 0, x, hb);
    set_vec(v, 1, y, hb);
    v.partials = (double *)c->buf[S_PARTIALS];
    v.part_stride = F.stride;
    HIP_TRY(blas_dot(prec, v, 2, F.s));
    return reduce_to_host(c, 2, F.stride, blas_blocks(v.n) * 2, out, F.s);
}

static wl_status norm_full(Fields &F, int prec, const void *x, double *out) {
    wl_ctx *c = F.c;
    VecArgs v = vec_args(c, prec, 1);
    set_vec(v, 0, x, half_bytes(c, prec, 1));
    v.partials = (double *)c->buf[S_PARTIALS];
    v.part_stride = F.stride;
    HIP_TRY(blas_norm2(prec, v, 2, F.s));
    return reduce_to_host(c, 1, F.stride, blas_blocks(v.n) * 2, out, F.s);
}

static wl_status caxpy_full(Fields &F, int prec, double ar, double ai, const void *x, void *y) {
    VecArgs v = vec_args(F.c, prec, 1);
    const size_t hb = half_bytes(F.c, prec, 1);
    set_vec(v, 0, x, hb);
    set_vec(v, 1, y, hb);
    v.a = ar;
    v.b = ai;
    HIP_TRY(blas_caxpy(prec, v, 2, F.s));
    return WL_OK;
}

// r = b - D x in FP64 (t: FP64 FULL temporary); *rn2 = ||r||^2
static wl_status system_residual(Fields &F, double kappa, const void *x, const void *b, void *r, void *t, double *rn2) {
    wl_ctx *c = F.c;
    wl_status st = apply_m(c, WL_OP_D, false, kappa, WL_F64, 18, 1, t, x, nullptr, nullptr, 0, nullptr, F.s, nullptr);
    if (st) return st;
    VecArgs v = vec_args(c, WL_F64, 1);
    const size_t hb = half_bytes(c, WL_F64, 1);
    set_vec(v, 0, b, hb);
    set_vec(v, 1, t, hb);
    set_vec(v, 2, r, hb);
    v.partials = (double *)c->buf[S_PARTIALS];
    v.part_stride = F.stride;
    HIP_TRY(blas_residual(WL_F64, v, 2, F.s));
    return reduce_to_host(c, 1, F.stride, blas_blocks(v.n) * 2, rn2, F.s);
}

extern "C" void wl_fgcr_params_default(wl_fgcr_params *p) {
    if (!p) return;
    p->tol = 1e-10;
    p->maxiter = 5000;
    p->restart = 16;
    p->fallback = 1;
    p->stagnation = 0.999;
}

extern "C" wl_status wl_cgnr_solve(wl_ctx *c, void *x, const void *eta, double kappa, const wl_solver_params *params,
                                   wl_solver_info *info, void *stream) {
    g_err.clear();
    const auto t0 = std::chrono::steady_clock::now();
    wl_status st = check_field_args(c, WL_FULL, WL_F64, 1);
    if (st) return st;
    if (!x || !eta || !aligned16(x) || !aligned16(eta)) return fail(WL_ERR_ARG, "null or misaligned field pointer");
    wl_solver_params P;
    wl_solver_params_default(&P);
    if (params) P = *params;
    if (!(P.tol > 0.0)) return fail(WL_ERR_ARG, "tolerance must be positive");
    Fields F{c, (hipStream_t)stream, part_stride_for(c, 1)};
    const size_t full = 2 * half_bytes(c, WL_F64, 1);
    if (overlap(x, full, eta, full)) return fail(WL_ERR_ARG, "x and eta overlap");
    if ((st = ensure_buf(c, S_GCR_R, full)) || (st = ensure_buf(c, S_GCR_TMP, full)) ||
        (st = ensure_buf(c, S_GCR_RHS, full)) || (st = ensure_buf(c, S_PARTIALS, sizeof(double) * 2 * F.stride)))
        return st;
    // rhs = D^+ eta
    if ((st = apply_m(c, WL_OP_D, true, kappa, WL_F64, 18, 1, c->buf[S_GCR_RHS], eta, nullptr, nullptr, 0, nullptr, F.s,
                      nullptr)))
        return st;
    double e2 = 0.0;
    if ((st = norm_full(F, WL_F64, eta, &e2))) return st;
    wl_solver_info acc{};
    double tol_n = P.tol;
    wl_status result = WL_NOT_CONVERGED;
    int rounds = 0;
    double rel = 0.0;
    for (;;) {
        wl_solver_params Q = P;
        Q.tol = tol_n;
        Q.maxiter = P.maxiter - acc.iters;
        wl_solver_info inf{};
        wl_status cs = wl_cg_solve(c, x, c->buf[S_GCR_RHS], WL_OP_D, kappa, 1, &Q, &inf, stream);
        if (cs < 0) return cs;
        acc.iters += inf.iters;
        acc.reliable_updates += inf.reliable_updates;
        acc.restarts += inf.restarts;
        double r2 = 0.0;
        if ((st = system_residual(F, kappa, x, eta, c->buf[S_GCR_R], c->buf[S_GCR_TMP], &r2))) return st;
        rel = e2 > 0 ? std::sqrt(r2 / e2) : 0.0;
        ++rounds;
        if (rel <= P.tol) {
            result = WL_OK;
            break;
        }
        if (cs == WL_BREAKDOWN) {
            result = WL_BREAKDOWN;
            break;
        }
        if (acc.iters >= P.maxiter || rounds > 8) break;
        // the normal-equation residual was met but the system residual was not: tighten
        tol_n *= std::max(1e-3, std::min(0.5, 0.5 * P.tol / rel));
    }
    acc.rel_resid = rel;
    acc.true_rel_resid = rel;
    acc.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (info) *info = acc;
    if (result == WL_NOT_CONVERGED) fail(WL_NOT_CONVERGED, "CGNR did not reach the system tolerance");
    return result;
}

// M^+ of the two-layer network: layer-2 adjoint (1 -> C channels), then layer-1 adjoint (C -> 1)
static wl_status ptc_adjoint_apply(wl_ctx *c, const wl_ptc *n, void *out, const void *in, void *hidden,
                                   hipStream_t s) {
    wl_status st;
    PtcArgs a2 = ptc_args(c, hidden, in, n->channels, 1, n->wb + 2 * n->n1, 1, &st);
    if (st) return st;
    HIP_TRY(launch_ptc_layer(a2, true, s));
    PtcArgs a1 = ptc_args(c, out, hidden, 1, n->channels, n->wb, 1, &st);
    if (st) return st;
    HIP_TRY(launch_ptc_layer(a1, true, s));
    return WL_OK;
}

extern "C" void wl_pcgnr_params_default(wl_pcgnr_params *p) {
    if (!p) return;
    p->tol = 1e-10;
    p->maxiter = 20000;
    p->inner_tol = 1e-5;
    p->fallback = 1;
    p->stagnation = 0.5;
}

extern "C" wl_status wl_pcgnr_solve(wl_ctx *c, void *x, const void *b, double kappa, const wl_ptc *net,
                                    const wl_pcgnr_params *params, wl_solver_info *info, void *stream) {
    g_err.clear();
    const auto t0 = std::chrono::steady_clock::now();
    wl_status st = check_field_args(c, WL_FULL, WL_F64, 1);
    if (st) return st;
    if (!x || !b || !aligned16(x) || !aligned16(b)) return fail(WL_ERR_ARG, "null or misaligned field pointer");
    wl_pcgnr_params P;
    wl_pcgnr_params_default(&P);
    if (params) P = *params;
    if (!(P.tol > 0.0) || P.maxiter < 1 || !(P.inner_tol > 0.0 && P.inner_tol < 1.0) ||
        !(P.stagnation > 0.0 && P.stagnation <= 1.0))
        return fail(WL_ERR_ARG, "bad preconditioned CGNR parameters");
    if (!std::isfinite(kappa)) return fail(WL_ERR_ARG, "non-finite kappa");
    Fields F{c, (hipStream_t)stream, part_stride_for(c, 1)};
    const size_t full_hi = 2 * half_bytes(c, WL_F64, 1), full_lo = 2 * half_bytes(c, WL_F32, 1);
    const size_t hb_lo = half_bytes(c, WL_F32, 1), hb_hi = half_bytes(c, WL_F64, 1);
    if (overlap(x, full_hi, b, full_hi)) return fail(WL_ERR_ARG, "x and b overlap");
    if ((st = ensure_buf(c, S_GCR_R, full_hi)) || (st = ensure_buf(c, S_GCR_TMP, full_hi)) ||
        (st = ensure_buf(c, S_PCG, 6 * full_lo)) || (st = ensure_buf(c, S_PARTIALS, sizeof(double) * 2 * F.stride)))
        return st;
    if (net && (st = ensure_buf(c, S_PTC_H, ptc_field_bytes(c, net->channels)))) return st;
    char *base = (char *)c->buf[S_PCG];
    void *y = base, *p = base + full_lo, *rho = base + 2 * full_lo, *sv = base + 3 * full_lo,
         *q = base + 4 * full_lo, *t = base + 5 * full_lo;
    void *rhi = c->buf[S_GCR_R], *thi = c->buf[S_GCR_TMP], *hid = net ? c->buf[S_PTC_H] : nullptr;
    // field-wide FP32 helpers (both parities)
    auto axpby = [&](double a, const void *v0, double bb, void *v1, double *n2) -> wl_status {
        VecArgs v = vec_args(c, WL_F32, 1);
        set_vec(v, 0, v0, hb_lo);
        set_vec(v, 1, v1, hb_lo);
        v.a = a;
        v.b = bb;
        v.partials = (double *)c->buf[S_PARTIALS];
        v.part_stride = F.stride;
        HIP_TRY(blas_axpby(WL_F32, v, 2, n2 != nullptr, F.s));
        if (n2) return reduce_to_host(c, 1, F.stride, blas_blocks(v.n) * 2, n2, F.s);
        return WL_OK;
    };
    auto copy_lo = [&](void *dst, const void *src) -> wl_status {
        VecArgs v = vec_args(c, WL_F32, 1);
        set_vec(v, 0, src, hb_lo);
        set_vec(v, 1, dst, hb_lo);
        HIP_TRY(blas_convert(WL_F32, WL_F32, false, v, 2, F.s));
        return WL_OK;
    };
    // out = M in (the network, or a copy when there is none)
    auto apply_net = [&](void *out, const void *in, bool adjoint) -> wl_status {
        if (!net) return copy_lo(out, in);
        return adjoint ? ptc_adjoint_apply(c, net, out, in, hid, F.s) : ptc_forward(c, net, out, in, hid, F.s);
    };
    double b2 = 0.0;
    if ((st = norm_full(F, WL_F64, b, &b2))) return st;
    wl_solver_info out{};
    if (!(b2 > 0.0)) {
        VecArgs v = vec_args(c, WL_F64, 1);
        set_vec(v, 0, x, hb_hi);
        HIP_TRY(blas_zero(WL_F64, v, 2, F.s));
        HIP_TRY(hipStreamSynchronize(F.s));
        if (info) *info = out;
        return WL_OK;
    }
    double rn2 = 0.0;
    if ((st = system_residual(F, kappa, x, b, rhi, thi, &rn2))) return st;
    const double target2 = P.tol * P.tol * b2;
    int total = 0, cycles = 0, stagnant = 0;
    bool failed = false;
    double rho2 = rn2;
    while (rn2 > target2) {
        if (total >= P.maxiter || !std::isfinite(rn2)) {
            failed = true;
            break;
        }
        // inner CG on the normal equations of (D M) y = r, FP32 fields, from y = 0
        {
            VecArgs v = vec_args(c, WL_F32, 1);
            set_vec(v, 0, rhi, hb_hi);
            set_vec(v, 1, rho, hb_lo);
            HIP_TRY(blas_convert(WL_F32, WL_F64, false, v, 2, F.s));
            set_vec(v, 0, y, hb_lo);
            HIP_TRY(blas_zero(WL_F32, v, 2, F.s));
        }
        const double start2 = rn2, stop2 = std::max(P.inner_tol * P.inner_tol * start2, 0.25 * target2);
        // s = M^+ D^+ rho, p = s
        if ((st = apply_m(c, WL_OP_D, true, kappa, WL_F32, 18, 1, t, rho, nullptr, nullptr, 0, nullptr, F.s, nullptr)) ||
            (st = apply_net(sv, t, true)) || (st = copy_lo(p, sv)))
            return st;
        double gam = 0.0;
        if ((st = norm_full(F, WL_F32, sv, &gam))) return st;
        bool breakdown = !(gam > 0.0) || !std::isfinite(gam);
        rho2 = start2;
        while (!breakdown && total < P.maxiter) {
            // q = D M p, ||q||^2 fused into the operator's epilogue
            if ((st = apply_net(t, p, false))) return st;
            double q2 = 0.0;
            {
                long nblk = 0;
                if ((st = apply_m(c, WL_OP_D, false, kappa, WL_F32, 18, 1, q, t, nullptr, (double *)c->buf[S_PARTIALS],
                                  F.stride, nullptr, F.s, &nblk)))
                    return st;
                if ((st = reduce_to_host(c, 1, F.stride, nblk, &q2, F.s))) return st;
            }
            if (!(q2 > 0.0) || !std::isfinite(q2)) {
                breakdown = true;
                break;
            }
            const double alpha = gam / q2;
            if ((st = axpby(alpha, p, 1.0, y, nullptr)) || (st = axpby(-alpha, q, 1.0, rho, &rho2))) return st;
            ++total;
            if (!std::isfinite(rho2)) {
                breakdown = true;
                break;
            }
            if (rho2 <= stop2) break;
            if ((st = apply_m(c, WL_OP_D, true, kappa, WL_F32, 18, 1, t, rho, nullptr, nullptr, 0, nullptr, F.s,
                              nullptr)) ||
                (st = apply_net(sv, t, true)))
                return st;
            double gam1 = 0.0;
            if ((st = norm_full(F, WL_F32, sv, &gam1))) return st;
            if (!std::isfinite(gam1)) {
                breakdown = true;
                break;
            }
            if ((st = axpby(1.0, sv, gam1 / gam, p, nullptr))) return st;
            gam = gam1;
        }
        // x += M y in FP64, then the FP64 residual
        if ((st = apply_net(t, y, false))) return st;
        {
            VecArgs v = vec_args(c, WL_F64, 1);
            set_vec(v, 0, t, hb_lo);
            set_vec(v, 1, x, hb_hi);
            HIP_TRY(blas_convert(WL_F64, WL_F32, true, v, 2, F.s));
        }
        const double prev = rn2;
        if ((st = system_residual(F, kappa, x, b, rhi, thi, &rn2))) return st;
        ++cycles;
        if (breakdown || !std::isfinite(rn2)) {
            failed = rn2 > target2 || !std::isfinite(rn2);
            break;
        }
        if (rn2 > P.stagnation * P.stagnation * prev) {
            if (++stagnant >= 2) {
                failed = true;
                break;
            }
        } else {
            stagnant = 0;
        }
    }
    out.iters = total;
    out.restarts = cycles;
    out.rel_resid = std::sqrt(rho2 / b2);
    out.true_rel_resid = std::sqrt(rn2 / b2);
    wl_status result = failed ? WL_NOT_CONVERGED : WL_OK;
    if (failed && P.fallback) {
        wl_solver_params Q;
        wl_solver_params_default(&Q);
        Q.tol = P.tol;
        wl_solver_info fi{};
        wl_status fs = wl_cgnr_solve(c, x, b, kappa, &Q, &fi, stream);
        if (fs < 0) return fs;
        out.fallback = 1;
        out.fallback_iters = fi.iters;
        out.true_rel_resid = fi.true_rel_resid;
        result = fs;
    }
    out.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (info) *info = out;
    if (result == WL_NOT_CONVERGED) fail(WL_NOT_CONVERGED, "preconditioned CGNR did not reach the tolerance");
    return result;
}

extern "C" wl_status wl_fgcr_solve(wl_ctx *c, void *x, const void *b, double kappa, const wl_ptc *net,
                                   const wl_fgcr_params *params, wl_solver_info *info, void *stream) {
    g_err.clear();
    const auto t0 = std::chrono::steady_clock::now();
    wl_status st = check_field_args(c, WL_FULL, WL_F64, 1);
    if (st) return st;
    if (!x || !b || !aligned16(x) || !aligned16(b)) return fail(WL_ERR_ARG, "null or misaligned field pointer");
    wl_fgcr_params P;
    wl_fgcr_params_default(&P);
    if (params) P = *params;
    if (!(P.tol > 0.0) || P.restart < 1 || P.restart > 64 || P.maxiter < 1) return fail(WL_ERR_ARG, "bad FGCR parameters");
    if (!std::isfinite(kappa)) return fail(WL_ERR_ARG, "non-finite kappa");
    const int m = P.restart;
    Fields F{c, (hipStream_t)stream, part_stride_for(c, 1)};
    const size_t full_hi = 2 * half_bytes(c, WL_F64, 1), full_lo = 2 * half_bytes(c, WL_F32, 1);
    if (overlap(x, full_hi, b, full_hi)) return fail(WL_ERR_ARG, "x and b overlap");
    if ((st = ensure_buf(c, S_GCR_R, full_hi)) || (st = ensure_buf(c, S_GCR_TMP, full_hi)) ||
        (st = ensure_buf(c, S_GCR_X, 2 * full_lo)) || (st = ensure_buf(c, S_GCR_Z, (size_t)m * full_lo)) ||
        (st = ensure_buf(c, S_GCR_W, (size_t)m * full_lo)) ||
        (st = ensure_buf(c, S_PARTIALS, sizeof(double) * 2 * F.stride)))
        return st;
    if (net && (st = ensure_buf(c, S_PTC_H, ptc_field_bytes(c, net->channels)))) return st;
    char *rlo = (char *)c->buf[S_GCR_X], *xc = rlo + full_lo;
    char *Z = (char *)c->buf[S_GCR_Z], *Wv = (char *)c->buf[S_GCR_W];
    void *rhi = c->buf[S_GCR_R], *thi = c->buf[S_GCR_TMP];
    double b2 = 0.0;
    if ((st = norm_full(F, WL_F64, b, &b2))) return st;
    wl_solver_info out{};
    if (!(b2 > 0.0)) {
        VecArgs v = vec_args(c, WL_F64, 1);
        set_vec(v, 0, x, half_bytes(c, WL_F64, 1));
        HIP_TRY(blas_zero(WL_F64, v, 2, F.s));
        HIP_TRY(hipStreamSynchronize(F.s));
        if (info) *info = out;
        return WL_OK;
    }
    double rn2 = 0.0;
    if ((st = system_residual(F, kappa, x, b, rhi, thi, &rn2))) return st;
    const double target2 = P.tol * P.tol * b2;
    int total = 0, cycles = 0, stagnant = 0;
    bool failed = false;
    std::vector<double> ww(m);
    double rlo2 = rn2;
    while (rn2 > target2) {
        if (total >= P.maxiter || !std::isfinite(rn2)) {
            failed = true;
            break;
        }
        // inner cycle in FP32 on the correction: D e = r
        {
            VecArgs v = vec_args(c, WL_F32, 1);
            const size_t hb = half_bytes(c, WL_F32, 1);
            set_vec(v, 0, rhi, half_bytes(c, WL_F64, 1));
            set_vec(v, 1, rlo, hb);
            HIP_TRY(blas_convert(WL_F32, WL_F64, false, v, 2, F.s));
            set_vec(v, 0, xc, hb);
            HIP_TRY(blas_zero(WL_F32, v, 2, F.s));
        }
        bool breakdown = false;
        for (int k = 0; k < m && total < P.maxiter; ++k) {
            void *zk = Z + (size_t)k * full_lo, *wk = Wv + (size_t)k * full_lo;
            if (net) {
                if ((st = ptc_forward(c, net, zk, rlo, c->buf[S_PTC_H], F.s))) return st;
            } else {
                VecArgs v = vec_args(c, WL_F32, 1);
                const size_t hb = half_bytes(c, WL_F32, 1);
                set_vec(v, 0, rlo, hb);
                set_vec(v, 1, zk, hb);
                HIP_TRY(blas_convert(WL_F32, WL_F32, false, v, 2, F.s));
            }
            if ((st = apply_m(c, WL_OP_D, false, kappa, WL_F32, 18, 1, wk, zk, nullptr, nullptr, 0, nullptr, F.s, nullptr)))
                return st;
            // modified Gram-Schmidt of w_k against the kept w_j (same combination on z_k)
            for (int j = 0; j < k; ++j) {
                void *zj = Z + (size_t)j * full_lo, *wj = Wv + (size_t)j * full_lo;
                double d[2];
                if ((st = dot_full(F, WL_F32, wj, wk, d))) return st;
                const double br = d[0] / ww[j], bi = d[1] / ww[j];
                if ((st = caxpy_full(F, WL_F32, -br, -bi, wj, wk)) || (st = caxpy_full(F, WL_F32, -br, -bi, zj, zk)))
                    return st;
            }
            if ((st = norm_full(F, WL_F32, wk, &ww[k]))) return st;
            if (!(ww[k] > 0.0) || !std::isfinite(ww[k])) {
                breakdown = true;
                break;
            }
            double d[2];
            if ((st = dot_full(F, WL_F32, wk, rlo, d))) return st;
            const double ar = d[0] / ww[k], ai = d[1] / ww[k];
            if ((st = caxpy_full(F, WL_F32, ar, ai, zk, xc)) || (st = caxpy_full(F, WL_F32, -ar, -ai, wk, rlo))) return st;
            if ((st = norm_full(F, WL_F32, rlo, &rlo2))) return st;
            ++total;
            if (!std::isfinite(rlo2)) {
                breakdown = true;
                break;
            }
            // the FP32 iterated residual cannot certify the tolerance: leave the
            // cycle a little below it and let the FP64 residual decide
            if (rlo2 <= 0.25 * target2) break;
        }
        // x += correction (FP64), then the FP64 residual
        {
            VecArgs v = vec_args(c, WL_F64, 1);
            set_vec(v, 0, xc, half_bytes(c, WL_F32, 1));
            set_vec(v, 1, x, half_bytes(c, WL_F64, 1));
            HIP_TRY(blas_convert(WL_F64, WL_F32, true, v, 2, F.s));
        }
        double prev = rn2;
        if ((st = system_residual(F, kappa, x, b, rhi, thi, &rn2))) return st;
        ++cycles;
        if (breakdown || !std::isfinite(rn2)) {
            failed = true;
            break;
        }
        if (rn2 > P.stagnation * P.stagnation * prev) {
            if (++stagnant >= 2) {
                failed = true;
                break;
            }
        } else {
            stagnant = 0;
        }
    }
    out.iters = total;
    out.restarts = cycles;
    out.rel_resid = std::sqrt(rlo2 / b2);
    out.true_rel_resid = std::sqrt(rn2 / b2);
    wl_status result = failed ? WL_NOT_CONVERGED : WL_OK;
    if (failed && P.fallback) {
        // plain FP64 CG on the normal equations, from the current x, judged on the same system residual
        wl_solver_params Q;
        wl_solver_params_default(&Q);
        Q.tol = P.tol;
        wl_solver_info fi{};
        wl_status fs = wl_cgnr_solve(c, x, b, kappa, &Q, &fi, stream);
        if (fs < 0) return fs;
        out.fallback = 1;
        out.fallback_iters = fi.iters;
        out.true_rel_resid = fi.true_rel_resid;
        result = fs;
    }
    out.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (info) *info = out;
    if (result == WL_NOT_CONVERGED) fail(WL_NOT_CONVERGED, "FGCR did not reach the tolerance");
    return result;
}
