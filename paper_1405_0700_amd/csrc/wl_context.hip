// C ABI, context layer: errors, the context (gauge copies, workspace), layout
// conversion kernels, timing and launch configuration.
#include "wl_internal.h"

// ------------------------------------------------------------------ errors
thread_local std::string wli::g_err;

wl_status wli::fail(wl_status st, const char *fmt, ...) {
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

wl_status wli::ensure_buf(wl_ctx *c, int slot, size_t bytes) {
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

wl_status wli::ensure_pinned(wl_ctx *c, size_t bytes) {
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
    // the allocation-free entry points' scratch address on this device (once per device)
    if (wl_status sst = scratch_setup(device)) return sst;
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
    g.f_lxh = make_fastdiv(g.lxh);
    g.f_ly = make_fastdiv(dims[1]);
    g.f_lz = make_fastdiv(dims[2]);
    g.f_sz = make_fastdiv(g.sz);
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
    // measured defaults (MI355X, 24^3x48 and 32^3x64 lattices): two threads per point;
    // FP64 blocks of 128 threads, FP32 blocks of 256 (2 % faster than 128 at 1, 4 and 12 rhs)
    c->cfg[WL_F64] = {128, 1, 2, WL_TCHUNK_AUTO, -1};
    c->cfg[WL_F32] = {256, 1, 2, WL_TCHUNK_AUTO, -1};
    // 16-bit storage: few registers per thread, so without a cap so many waves are in flight
    // that their neighbour spinors crowd each other out of L2; about 4 waves per SIMD measured
    // best (FP16 half-dslash at 32^3x64: 82 -> 67 us)
    c->cfg[WL_F16N] = {256, 1, 1, WL_TCHUNK_AUTO, -1, 1, 0, 4};
    c->cfg[WL_BF16N] = {256, 1, 1, WL_TCHUNK_AUTO, -1, 1, 0, 4};
    c->cfg[WL_I16N] = {256, 1, 1, WL_TCHUNK_AUTO, -1, 1, 0, 4};
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

wl_status wli::get_links(wl_ctx *c, int prec, int recon, const void **ptr, size_t *slab) {
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

VecArgs wli::vec_args(const wl_ctx *c, int prec, int nrhs) {
    VecArgs a;
    std::memset(&a, 0, sizeof a);
    a.n = c->Vh * (long)nrhs;
    a.nrhs = nrhs;
    (void)prec;
    return a;
}
void wli::set_vec(VecArgs &a, int k, const void *base, size_t hb) {
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

const char *wli::launch_problem(int block, int tps, int nt, int rpt, int occ, int sweep) {
    if (block < 64 || block > 256 || block % 64) return "block not in {64, 128, 192, 256}";
    if (occ < 0 || occ > 8) return "occ not in 0..8";
    if (sweep < 0 || sweep > 65536) return "sweep not in 0..65536";
    if (tps != 1 && tps != 2) return "tps not in {1, 2}";
    if (nt < -1 || nt > 1) return "nt not in {-1, 0, 1}";
    if (rpt < 1 || rpt > 4) return "rpt not in 1..4";
    if (rpt > 1 && tps != 1) return "rpt > 1 needs tps = 1";
    return nullptr;
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
    if (const char *why = launch_problem(l->block, l->tps, l->nt, l->rpt, l->occ, l->sweep))
        return fail(WL_ERR_ARG, "launch (block %d, tps %d, nt %d, rpt %d, occ %d, sweep %d): %s", l->block, l->tps,
                    l->nt, l->rpt, l->occ, l->sweep, why);
    LaunchCfg &g = c->cfg[prec];
    g.block = l->block;
    g.swizzle = l->swizzle ? 1 : 0;
    g.tps = l->tps;
    g.tchunk = l->tchunk;
    g.nt = l->nt;
    g.rpt = l->rpt;
    g.occ = l->occ;
    g.sweep = l->sweep;
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
    l->occ = g.occ;
    l->sweep = g.sweep;
    return WL_OK;
}
