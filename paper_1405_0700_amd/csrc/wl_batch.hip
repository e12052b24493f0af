// C ABI, batch layer: several lattices in lockstep with one persistent launch
// per hopping stage, and the launch autotuners.
#include "wl_internal.h"

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
                    for (int tch : {0, 4, WL_TCHUNK_AUTO, WL_TCHUNK_YZ})
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
        chosen->occ = best.occ;
        chosen->sweep = best.sweep;
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
