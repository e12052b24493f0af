// C ABI, learned-preconditioner layer: the PTC network (forward, adjoint,
// gradients, Adam) and the solvers that use it (FGCR, CG on D M) with plain
// FP64 CGNR as comparison and fallback.
#include "wl_internal.h"

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
    uint16_t *tab = nullptr;  // matrix-core operand tables (forward, then adjoint) of the BF16 weights
    mutable bool tab_ok = false;  // false until built, and again after every weight update
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
        (e = hipMalloc(&n->v, nr * sizeof(float))) != hipSuccess || (e = hipMalloc(&n->loss, sizeof(double))) != hipSuccess ||
        (ptc_net_supported(channels) &&
         (e = hipMalloc(&n->tab, 2 * ptc_net_table_elems(channels) * sizeof(uint16_t))) != hipSuccess)) {
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
    if (n->tab) (void)hipFree(n->tab);
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

extern "C" wl_status wl_ptc_get_moments(const wl_ptc *n, double *m1, double *m2, double *v1, double *v2) {
    g_err.clear();
    if (!n) return fail(WL_ERR_ARG, "null network");
    HIP_TRY(hipDeviceSynchronize());
    wl_status st = ptc_download(n, n->m, false, m1, m2);
    if (st) return st;
    return ptc_download(n, n->v, false, v1, v2);
}

// bytes of a C-channel PTC field: C consecutive FULL FP32 single-rhs fields
static size_t ptc_field_bytes(const wl_ctx *c, int channels, int nrhs = 1) {
    return (size_t)channels * 2 * half_bytes(c, WL_F32, nrhs);
}

static PtcArgs ptc_args(wl_ctx *c, void *out, const void *in, int cout, int cin, const void *w, int adjoint,
                        wl_status *st, int nrhs = 1) {
    PtcArgs a;
    std::memset(&a, 0, sizeof a);
    const void *gauge = nullptr;
    size_t slab = 0;
    *st = get_links(c, WL_F32, 18, &gauge, &slab);
    a.g = c->g;
    (void)cin;
    a.out = (char *)out;
    a.in = (const char *)in;
    a.half = half_bytes(c, WL_F32, nrhs);
    a.gauge = gauge;
    a.slab_bytes = slab;
    a.w = w;
    a.cout = cout;
    a.cin = cin;
    a.adjoint = adjoint;
    a.vh = c->Vh;
    a.nrhs = nrhs;
    return a;
}

// out = M(in) = layer2(layer1(in)) with the BF16 weights; the hidden field is
// returned in `hidden` (channels C)
static wl_status ptc_adjoint_apply(wl_ctx *c, const wl_ptc *n, void *out, const void *in, void *hidden,
                                   hipStream_t s, int nrhs);
// the nine path fields of a one-output-channel layer's two-pass form (nrhs right-hand sides)
static wl_status ptc_paths(wl_ctx *c, int nrhs, char **paths) {
    wl_status st = ensure_buf(c, S_PTC_PATHS, (size_t)PTC_NPATH * 2 * half_bytes(c, WL_F32, nrhs));
    *paths = st ? nullptr : (char *)c->buf[S_PTC_PATHS];
    return st;
}
// out = M in for nrhs right-hand sides (FULL FP32 fields of nrhs; hidden: channels times that)
static wl_status ptc_forward(wl_ctx *c, const wl_ptc *n, void *out, const void *in, void *hidden, hipStream_t s,
                             int nrhs = 1) {
    wl_status st;
    char *paths = nullptr;
    if ((st = ptc_paths(c, nrhs, &paths))) return st;
    PtcArgs a1 = ptc_args(c, hidden, in, n->channels, 1, n->wb, 0, &st, nrhs);
    if (st) return st;
    HIP_TRY(launch_ptc_layer(a1, true, s));
    PtcArgs a2 = ptc_args(c, out, hidden, 1, n->channels, n->wb + 2 * n->n1, 0, &st, nrhs);
    a2.paths = paths;
    if (st) return st;
    HIP_TRY(launch_ptc_layer(a2, true, s));
    return WL_OK;
}

// out = M in (adjoint: M^+ in) for nrhs right-hand sides, without the hidden field: the
// matrix-core network for 4 or 8 channels, else the layer kernels with the hidden field in S_PTC_H
static wl_status ptc_net_apply(wl_ctx *c, const wl_ptc *n, void *out, const void *in, bool adjoint, hipStream_t s,
                               int nrhs) {
    wl_status st;
    if (!n->tab) {
        if ((st = ensure_buf(c, S_PTC_H, ptc_field_bytes(c, n->channels, nrhs)))) return st;
        return adjoint ? ptc_adjoint_apply(c, n, out, in, c->buf[S_PTC_H], s, nrhs)
                       : ptc_forward(c, n, out, in, c->buf[S_PTC_H], s, nrhs);
    }
    const long te = ptc_net_table_elems(n->channels);
    if (!n->tab_ok) {
        HIP_TRY(launch_ptc_net_tables(n->wb, n->n1, n->channels, n->tab, n->tab + te, s));
        n->tab_ok = true;
    }
    char *paths = nullptr;
    if ((st = ptc_paths(c, nrhs, &paths))) return st;
    PtcArgs a = ptc_args(c, out, in, 1, 1, nullptr, adjoint ? 1 : 0, &st, nrhs);
    if (st) return st;
    a.paths = paths;
    HIP_TRY(launch_ptc_net(a, n->channels, n->tab + (adjoint ? te : 0), s));
    return WL_OK;
}

extern "C" wl_status wl_ptc_apply(wl_ctx *c, const wl_ptc *n, void *out, const void *in, int nrhs, int adjoint,
                                  void *stream) {
    g_err.clear();
    if (!c || !n || !out || !in || !aligned16(out) || !aligned16(in)) return fail(WL_ERR_ARG, "null or misaligned argument");
    if (nrhs < 1 || nrhs > 64) return fail(WL_ERR_ARG, "nrhs %d outside [1, 64]", nrhs);
    const size_t hb = half_bytes(c, WL_F32, nrhs);
    if (overlap(out, 2 * hb, in, 2 * hb)) return fail(WL_ERR_ARG, "out and in overlap");
    return ptc_net_apply(c, n, out, in, adjoint != 0, (hipStream_t)stream, nrhs);
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
    n->tab_ok = false;
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

// ||x_r||^2 for every rhs of a FULL field of nrhs
static wl_status norms_full(Fields &F, int prec, const void *x, int nrhs, double *out) {
    wl_ctx *c = F.c;
    VecArgs v = vec_args(c, prec, nrhs);
    set_vec(v, 0, x, half_bytes(c, prec, nrhs));
    v.partials = (double *)c->buf[S_PARTIALS];
    v.part_stride = F.stride;
    HIP_TRY(blas_norm2(prec, v, 2, F.s));
    return reduce_to_host(c, nrhs, F.stride, blas_blocks(v.n) * 2, out, F.s);
}

// r = b - D x in FP64 for nrhs right-hand sides (t: FP64 FULL temporary); rn2[r] = ||r_r||^2
static wl_status system_residuals(Fields &F, double kappa, const void *x, const void *b, void *r, void *t, int nrhs,
                                  double *rn2) {
    wl_ctx *c = F.c;
    wl_status st =
        apply_m(c, WL_OP_D, false, kappa, WL_F64, 18, nrhs, t, x, nullptr, nullptr, 0, nullptr, F.s, nullptr);
    if (st) return st;
    VecArgs v = vec_args(c, WL_F64, nrhs);
    const size_t hb = half_bytes(c, WL_F64, nrhs);
    set_vec(v, 0, b, hb);
    set_vec(v, 1, t, hb);
    set_vec(v, 2, r, hb);
    v.partials = (double *)c->buf[S_PARTIALS];
    v.part_stride = F.stride;
    HIP_TRY(blas_residual(WL_F64, v, 2, F.s));
    return reduce_to_host(c, nrhs, F.stride, blas_blocks(v.n) * 2, rn2, F.s);
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

// Plain FP64 CG for D x = eta (reading C-7: every solver of D x = eta is stopped on the system residual
// ||eta - D x|| <= tol ||eta||): CG on D^+ D x = D^+ eta (wl_cg_solve), the normal-equation tolerance
// tightened and the CG continued from x until the FP64 system residual of every rhs meets tol.
extern "C" wl_status wl_cgnr_solve(wl_ctx *c, void *x, const void *eta, double kappa, int nrhs,
                                   const wl_solver_params *params, wl_solver_info *info, void *stream) {
    g_err.clear();
    const auto t0 = std::chrono::steady_clock::now();
    wl_status st = check_field_args(c, WL_FULL, WL_F64, nrhs);
    if (st) return st;
    if (!x || !eta || !aligned16(x) || !aligned16(eta)) return fail(WL_ERR_ARG, "null or misaligned field pointer");
    wl_solver_params P;
    wl_solver_params_default(&P);
    if (params) P = *params;
    if (!(P.tol > 0.0)) return fail(WL_ERR_ARG, "tolerance must be positive");
    Fields F{c, (hipStream_t)stream, part_stride_for(c, nrhs)};
    const size_t full = 2 * half_bytes(c, WL_F64, nrhs);
    if (overlap(x, full, eta, full)) return fail(WL_ERR_ARG, "x and eta overlap");
    if ((st = ensure_buf(c, S_GCR_R, full)) || (st = ensure_buf(c, S_GCR_TMP, full)) ||
        (st = ensure_buf(c, S_GCR_RHS, full)) ||
        (st = ensure_buf(c, S_PARTIALS, sizeof(double) * 2 * nrhs * F.stride)))
        return st;
    // rhs = D^+ eta
    if ((st = apply_m(c, WL_OP_D, true, kappa, WL_F64, 18, nrhs, c->buf[S_GCR_RHS], eta, nullptr, nullptr, 0,
                      nullptr, F.s, nullptr)))
        return st;
    std::vector<double> e2(nrhs), r2(nrhs), rel(nrhs, 0.0);
    if ((st = norms_full(F, WL_F64, eta, nrhs, e2.data()))) return st;
    std::vector<wl_solver_info> acc(nrhs);
    std::vector<wl_solver_info> inf(nrhs);
    double tol_n = P.tol;
    wl_status result = WL_NOT_CONVERGED;
    int rounds = 0, done_iters = 0;
    for (;;) {
        wl_solver_params Q = P;
        Q.tol = tol_n;
        Q.maxiter = P.maxiter - done_iters;
        wl_status cs = wl_cg_solve(c, x, c->buf[S_GCR_RHS], WL_OP_D, kappa, nrhs, &Q, inf.data(), stream);
        if (cs < 0) return cs;
        int most = 0;
        for (int r = 0; r < nrhs; ++r) {
            acc[r].iters += inf[r].iters;
            acc[r].reliable_updates += inf[r].reliable_updates;
            acc[r].restarts += inf[r].restarts;
            most = std::max(most, inf[r].iters);
        }
        done_iters += most;
        if ((st = system_residuals(F, kappa, x, eta, c->buf[S_GCR_R], c->buf[S_GCR_TMP], nrhs, r2.data()))) return st;
        double worst = 0.0;
        for (int r = 0; r < nrhs; ++r) {
            rel[r] = e2[r] > 0 ? std::sqrt(r2[r] / e2[r]) : 0.0;
            worst = std::max(worst, rel[r]);
        }
        ++rounds;
        if (worst <= P.tol) {
            result = WL_OK;
            break;
        }
        if (cs == WL_BREAKDOWN) {
            result = WL_BREAKDOWN;
            break;
        }
        if (done_iters >= P.maxiter || rounds > 8) break;
        // the normal-equation residual was met but the system residual was not: tighten
        tol_n *= std::max(1e-3, std::min(0.5, 0.5 * P.tol / worst));
    }
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    for (int r = 0; r < nrhs; ++r) {
        acc[r].rel_resid = rel[r];
        acc[r].true_rel_resid = rel[r];
        acc[r].seconds = secs;
        if (info) info[r] = acc[r];
    }
    if (result == WL_NOT_CONVERGED) fail(WL_NOT_CONVERGED, "CGNR did not reach the system tolerance");
    return result;
}

// M^+ of the two-layer network: layer-2 adjoint (1 -> C channels), then layer-1 adjoint (C -> 1)
static wl_status ptc_adjoint_apply(wl_ctx *c, const wl_ptc *n, void *out, const void *in, void *hidden,
                                   hipStream_t s, int nrhs) {
    wl_status st;
    PtcArgs a2 = ptc_args(c, hidden, in, n->channels, 1, n->wb + 2 * n->n1, 1, &st, nrhs);
    if (st) return st;
    HIP_TRY(launch_ptc_layer(a2, true, s));
    char *paths = nullptr;
    if ((st = ptc_paths(c, nrhs, &paths))) return st;
    PtcArgs a1 = ptc_args(c, out, hidden, 1, n->channels, n->wb, 1, &st, nrhs);
    a1.paths = paths;
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

// CG on the normal equations of the right-preconditioned system D M y = b, x = M y (reading R-20; the
// flexible / preconditioned solver of the learned-preconditioner workload, reading C-16), for nrhs
// right-hand sides sharing every operator and network application.  Inner cycle in FP32 on the
// correction of the FP64 residual with per-rhs scalars on the device (no host round trip per
// iteration); defect correction in FP64; stopped on the system residual (reading C-7).
extern "C" wl_status wl_pcgnr_solve(wl_ctx *c, void *x, const void *b, double kappa, const wl_ptc *net, int nrhs,
                                    const wl_pcgnr_params *params, wl_solver_info *info, void *stream) {
    g_err.clear();
    const auto t0 = std::chrono::steady_clock::now();
    wl_status st = check_field_args(c, WL_FULL, WL_F64, nrhs);
    if (st) return st;
    if (!x || !b || !aligned16(x) || !aligned16(b)) return fail(WL_ERR_ARG, "null or misaligned field pointer");
    wl_pcgnr_params P;
    wl_pcgnr_params_default(&P);
    if (params) P = *params;
    if (!(P.tol > 0.0) || P.maxiter < 1 || !(P.inner_tol > 0.0 && P.inner_tol < 1.0) ||
        !(P.stagnation > 0.0 && P.stagnation <= 1.0))
        return fail(WL_ERR_ARG, "bad preconditioned CGNR parameters");
    if (!std::isfinite(kappa)) return fail(WL_ERR_ARG, "non-finite kappa");
    Fields F{c, (hipStream_t)stream, part_stride_for(c, nrhs)};
    const size_t hb_lo = half_bytes(c, WL_F32, nrhs), hb_hi = half_bytes(c, WL_F64, nrhs);
    const size_t full_hi = 2 * hb_hi, full_lo = 2 * hb_lo;
    if (overlap(x, full_hi, b, full_hi)) return fail(WL_ERR_ARG, "x and b overlap");
    // device scalars: PcgScalars[nrhs], then the active count, then rho2_start / stop2 (doubles), live (ints)
    const size_t sc_bytes = sizeof(PcgScalars) * nrhs + 64 + sizeof(double) * 2 * nrhs + sizeof(int) * nrhs;
    if ((st = ensure_buf(c, S_GCR_R, full_hi)) || (st = ensure_buf(c, S_GCR_TMP, full_hi)) ||
        (st = ensure_buf(c, S_PCG, 6 * full_lo)) ||
        (st = ensure_buf(c, S_PARTIALS, sizeof(double) * 2 * nrhs * F.stride)) ||
        (st = ensure_buf(c, S_PCG_SC, sc_bytes)))
        return st;
    char *base = (char *)c->buf[S_PCG];
    void *y = base, *p = base + full_lo, *rho = base + 2 * full_lo, *sv = base + 3 * full_lo,
         *q = base + 4 * full_lo, *t = base + 5 * full_lo;
    void *rhi = c->buf[S_GCR_R], *thi = c->buf[S_GCR_TMP];
    PcgScalars *sc = (PcgScalars *)c->buf[S_PCG_SC];
    int *count = (int *)((char *)sc + sizeof(PcgScalars) * nrhs);
    double *d_start = (double *)((char *)count + 64), *d_stop = d_start + nrhs;
    int *d_live = (int *)(d_stop + nrhs);
    double *partials = (double *)c->buf[S_PARTIALS];
    auto convert = [&](int dp, void *dst, size_t dh, int sp, const void *src, size_t sh, bool acc) -> wl_status {
        VecArgs v = vec_args(c, dp, nrhs);
        set_vec(v, 0, src, sh);
        set_vec(v, 1, dst, dh);
        HIP_TRY(blas_convert(dp, sp, acc, v, 2, F.s));
        return WL_OK;
    };
    // out = M in (a copy without a network), for all rhs
    auto apply_net = [&](void *out, const void *in, bool adjoint) -> wl_status {
        if (!net) return convert(WL_F32, out, hb_lo, WL_F32, in, hb_lo, false);
        return ptc_net_apply(c, net, out, in, adjoint, F.s, nrhs);
    };
    // sv = M^+ D^+ rho and the partials of ||sv||^2 per rhs
    long nblk_blas = blas_blocks(c->Vh * (long)nrhs) * 2;
    auto normal_residual = [&]() -> wl_status {
        wl_status e =
            apply_m(c, WL_OP_D, true, kappa, WL_F32, 18, nrhs, t, rho, nullptr, nullptr, 0, nullptr, F.s, nullptr);
        if (e || (e = apply_net(sv, t, true))) return e;
        VecArgs v = vec_args(c, WL_F32, nrhs);
        set_vec(v, 0, sv, hb_lo);
        v.partials = partials;
        v.part_stride = F.stride;
        HIP_TRY(blas_norm2(WL_F32, v, 2, F.s));
        return WL_OK;
    };
    PcgVec pv;
    std::memset(&pv, 0, sizeof pv);
    pv.y[0] = y, pv.y[1] = (char *)y + hb_lo;
    pv.p[0] = p, pv.p[1] = (char *)p + hb_lo;
    pv.rho[0] = rho, pv.rho[1] = (char *)rho + hb_lo;
    pv.n = c->Vh * (long)nrhs;
    pv.nrhs = nrhs;
    pv.sc = sc;
    pv.partials = partials;
    pv.part_stride = F.stride;

    std::vector<double> b2(nrhs), rn2(nrhs), target2(nrhs), prev(nrhs);
    std::vector<int> done(nrhs, 0), failed(nrhs, 0), stagnant(nrhs, 0), live(nrhs, 0), zero(nrhs, 0);
    std::vector<wl_solver_info> out(nrhs);
    if ((st = norms_full(F, WL_F64, b, nrhs, b2.data()))) return st;
    bool any_zero = false;
    for (int r = 0; r < nrhs; ++r)
        if (!(b2[r] > 0.0)) zero[r] = 1, any_zero = true;
    if (any_zero) {
        // D x = 0: x = 0 for those right-hand sides
        HIP_TRY(hipMemcpyAsync(d_live, zero.data(), sizeof(int) * nrhs, hipMemcpyHostToDevice, F.s));
        HIP_TRY(blas_zero_masked(WL_F64, x, hb_hi, pv.n, nrhs, d_live, F.s));
    }
    if ((st = system_residuals(F, kappa, x, b, rhi, thi, nrhs, rn2.data()))) return st;
    for (int r = 0; r < nrhs; ++r) {
        target2[r] = P.tol * P.tol * b2[r];
        done[r] = zero[r] || rn2[r] <= target2[r];
    }
    int total = 0;  // inner iterations of the slowest rhs
    std::vector<PcgScalars> hs(nrhs);
    for (;;) {
        int nlive = 0;
        for (int r = 0; r < nrhs; ++r) {
            live[r] = !done[r] && !failed[r];
            nlive += live[r];
        }
        if (!nlive) break;
        if (total >= P.maxiter) {
            for (int r = 0; r < nrhs; ++r)
                if (live[r]) failed[r] = 1;
            break;
        }
        // a cycle: rho = r (FP32), y = 0, inner CG until every live rhs has dropped by inner_tol
        std::vector<double> stop2(nrhs);
        for (int r = 0; r < nrhs; ++r) stop2[r] = std::max(P.inner_tol * P.inner_tol * rn2[r], 0.25 * target2[r]);
        if ((st = convert(WL_F32, rho, hb_lo, WL_F64, rhi, hb_hi, false))) return st;
        {
            VecArgs v = vec_args(c, WL_F32, nrhs);
            set_vec(v, 0, y, hb_lo);
            HIP_TRY(blas_zero(WL_F32, v, 2, F.s));
        }
        HIP_TRY(hipMemcpyAsync(d_start, rn2.data(), sizeof(double) * nrhs, hipMemcpyHostToDevice, F.s));
        HIP_TRY(hipMemcpyAsync(d_stop, stop2.data(), sizeof(double) * nrhs, hipMemcpyHostToDevice, F.s));
        HIP_TRY(hipMemcpyAsync(d_live, live.data(), sizeof(int) * nrhs, hipMemcpyHostToDevice, F.s));
        HIP_TRY(hipMemsetAsync(count, 0, sizeof(int), F.s));
        if ((st = normal_residual())) return st;
        HIP_TRY(pcg_start(sc, nrhs, partials, F.stride, nblk_blas, d_start, d_stop, d_live, count, F.s));
        if ((st = convert(WL_F32, p, hb_lo, WL_F32, sv, hb_lo, false))) return st;
        int it = 0, still = 1;
        const int budget = P.maxiter - total;
        while (still && it < budget) {
            // a block of iterations on device scalars, then one read of the active count
            const int blk = std::min(8, budget - it);
            for (int k = 0; k < blk; ++k) {
                // q = D M p with ||q||^2 per rhs
                long nblk = 0;
                if ((st = apply_net(t, p, false)) ||
                    (st = apply_m(c, WL_OP_D, false, kappa, WL_F32, 18, nrhs, q, t, nullptr, partials, F.stride,
                                  nullptr, F.s, &nblk)))
                    return st;
                HIP_TRY(pcg_alpha(sc, nrhs, partials, F.stride, nblk, count, F.s));
                pv.q[0] = q, pv.q[1] = (char *)q + hb_lo;
                HIP_TRY(pcg_update_yr(pv, F.s));
                HIP_TRY(pcg_check(sc, nrhs, partials, F.stride, nblk_blas, count, F.s));
                if ((st = normal_residual())) return st;
                HIP_TRY(pcg_beta(sc, nrhs, partials, F.stride, nblk_blas, count, F.s));
                pv.q[0] = sv, pv.q[1] = (char *)sv + hb_lo;
                HIP_TRY(pcg_update_p(pv, F.s));
            }
            it += blk;
            HIP_TRY(hipMemcpyAsync(&still, count, sizeof(int), hipMemcpyDeviceToHost, F.s));
            HIP_TRY(hipStreamSynchronize(F.s));
        }
        HIP_TRY(hipMemcpyAsync(hs.data(), sc, sizeof(PcgScalars) * nrhs, hipMemcpyDeviceToHost, F.s));
        // x += M y in FP64, then the FP64 residual
        if ((st = apply_net(t, y, false)) || (st = convert(WL_F64, x, hb_hi, WL_F32, t, hb_lo, true))) return st;
        prev = rn2;
        if ((st = system_residuals(F, kappa, x, b, rhi, thi, nrhs, rn2.data()))) return st;
        int most = 0;
        for (int r = 0; r < nrhs; ++r) {
            if (!live[r]) continue;
            out[r].iters += hs[r].iters;
            out[r].restarts += 1;
            out[r].rel_resid = std::sqrt(hs[r].rho2 / b2[r]);
            most = std::max(most, hs[r].iters);
            if (rn2[r] <= target2[r]) {
                done[r] = 1;
            } else if (hs[r].breakdown || !std::isfinite(rn2[r])) {
                failed[r] = 1;
            } else if (rn2[r] > P.stagnation * P.stagnation * prev[r]) {
                if (++stagnant[r] >= 2) failed[r] = 1;
            } else {
                stagnant[r] = 0;
            }
        }
        total += std::max(most, 1);
    }
    wl_status result = WL_OK;
    bool any_failed = false;
    for (int r = 0; r < nrhs; ++r) {
        out[r].true_rel_resid = b2[r] > 0 ? std::sqrt(rn2[r] / b2[r]) : 0.0;
        any_failed = any_failed || failed[r];
    }
    if (any_failed) result = WL_NOT_CONVERGED;
    if (any_failed && P.fallback) {
        // plain FP64 CG continues every rhs from its x (those already converged need no iterations)
        wl_solver_params Q;
        wl_solver_params_default(&Q);
        Q.tol = P.tol;
        std::vector<wl_solver_info> fi(nrhs);
        wl_status fs = wl_cgnr_solve(c, x, b, kappa, nrhs, &Q, fi.data(), stream);
        if (fs < 0) return fs;
        for (int r = 0; r < nrhs; ++r) {
            if (failed[r]) {
                out[r].fallback = 1;
                out[r].fallback_iters = fi[r].iters;
            }
            out[r].true_rel_resid = fi[r].true_rel_resid;
        }
        result = fs;
    }
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    for (int r = 0; r < nrhs; ++r) {
        out[r].seconds = secs;
        if (info) info[r] = out[r];
    }
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
                if ((st = ptc_net_apply(c, net, zk, rlo, false, F.s, 1))) return st;
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
        wl_status fs = wl_cgnr_solve(c, x, b, kappa, 1, &Q, &fi, stream);
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
