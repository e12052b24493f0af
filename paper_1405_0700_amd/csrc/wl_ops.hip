// C ABI, operator layer: hopping term, Dirac operator and its Schur complement,
// even/odd helpers, BLAS-1 entry points and the link-spinor access kernel.
#include "wl_internal.h"

// ------------------------------------------------------------------ operators
// Enqueue out = a x + b H in (or H^+) for one output subset.
// HopArgs of out = a x + b H in for one output subset; *np = output parities
wl_status wli::fill_hop_args(wl_ctx *c, int prec, int recon, void *out, const void *in, const void *x,
                               int out_subset, int nrhs, double a, double b, double *partials, long part_stride,
                               const int *flag, HopArgs &h, int *np_out, double tm_x, double tm_h) {
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
void wli::set_cg_residual(const wl_ctx *c, int prec, int nrhs, int out_subset, void *cg_r, const CGScalars *cg_sc,
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

wl_status wli::hop_core(wl_ctx *c, int prec, int recon, bool dag, int epi, void *out, const void *in,
                          const void *x, int out_subset, int nrhs, double a, double b, double *partials,
                          long part_stride, const int *flag, hipStream_t s, long *nblk_out,
                          double tm_x, double tm_h, void *cg_r,
                          const CGScalars *cg_sc) {
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
    }
    const LaunchCfg &cfg = c->cfg[prec];
    HIP_TRY(launch_hop(prec, recon, dag, epi, h, np, cfg, s, ev ? ev[0] : nullptr, ev ? ev[1] : nullptr));
    if (nblk_out)
        *nblk_out = hop_launch_blocks(effective_tps(prec, cfg), cfg, h.npts, nrhs, h.g.L[3], h.g.st, prec) * np;
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
wl_status wli::apply_m(wl_ctx *c, int op, bool dag, double kappa, int prec, int recon, int nrhs, void *out,
                         const void *in, void *tmp, double *partials, long stride, const int *flag, hipStream_t s,
                         long *nblk, double mu) {
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
wl_status wli::apply_mdag_update_r(wl_ctx *c, int op, double kappa, int prec, int recon, int nrhs, void *r,
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
long wli::part_stride_for(const wl_ctx *c, int nrhs) {
    const long n = c->Vh * (long)nrhs;
    const long hb = hop_blocks(n, 64, 2) * 2;  // the most blocks any hopping launch may use
    const long sb = hop_blocks((long)c->g.st * nrhs, 64, 1) * c->g.L[3] * 2;  // time sweep, one slice per block
    const long bb = blas_blocks(n) * 2;
    return std::max(std::max(hb, sb), bb);
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

wl_status wli::reduce_to_host(wl_ctx *c, int nvals, long stride, long nblk, double *out, hipStream_t s) {
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
