// C ABI, CG layer: conjugate gradient on the normal equations (FP64 or mixed
// precision with FP64 reliable updates), multi-RHS, graph-captured iteration.
#include "wl_internal.h"

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
wl_status wli::true_residual(CGRun &R) {
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
wl_status wli::load_residual(CGRun &R) {
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
wl_status wli::cg_finish_iteration(CGRun &R, bool reliable) {
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

wl_status wli::cg_iteration(CGRun &R, bool reliable) {
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
std::vector<uintptr_t> wli::graph_key(const CGRun &R) {
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
wl_status wli::cg_setup(wl_ctx *c, void *x, const void *b, int op, double kappa, int nrhs, const wl_solver_params &P,
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
