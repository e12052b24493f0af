// C ABI, EigCG layer: incremental eigCG on the normal equations.
#include "wl_internal.h"

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
