// BLAS-1 steps of the solvers on internal spinor fields (gfx950).
//
// Each kernel streams whole spinor points (12 complex) with one thread per
// point; the reductions are accumulated in FP64, first per block (wavefront
// shuffles, then LDS, in a fixed order) into a partials array, then by a
// single-block kernel in a fixed order, so results are bitwise reproducible
// from run to run.
#include "wl_blas.h"

namespace wl {

#define WL_FLAG_EXIT \
    if (a.flag && *a.flag == 0) return;

template <int SP, bool NORM>
__global__ void __launch_bounds__(256) k_axpby(const VecArgs a) {
    using T = typename SpinorIO<SP>::real;
    WL_FLAG_EXIT
    const int h = blockIdx.y;
    const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
    double nrm = 0.0;
    if (gid < a.n) {
        cpx<T> x[12], y[12];
        SpinorIO<SP>::load(a.v[0][h], gid, x);
        SpinorIO<SP>::load(a.v[1][h], gid, y);
        const T aa = (T)a.a, bb = (T)a.b;
#pragma unroll
        for (int k = 0; k < 12; ++k) y[k] = {fma(aa, x[k].re, bb * y[k].re), fma(aa, x[k].im, bb * y[k].im)};
        SpinorIO<SP>::store(a.v[1][h], gid, y);
        if constexpr (NORM) {
            if constexpr (SP != WL_F64) SpinorIO<SP>::load(a.v[1][h], gid, y);
#pragma unroll
            for (int k = 0; k < 12; ++k) nrm += (double)y[k].re * y[k].re + (double)y[k].im * y[k].im;
        }
    }
    if constexpr (NORM) {
        __shared__ double lds[256];
        block_sum_rhs(nrm, gid, a.nrhs, lds, a.partials + (long)blockIdx.y * gridDim.x + blockIdx.x,
                      a.part_stride);
    }
}

template <int SP>
__global__ void __launch_bounds__(256) k_dot(const VecArgs a) {
    using T = typename SpinorIO<SP>::real;
    WL_FLAG_EXIT
    const int h = blockIdx.y;
    const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
    double re = 0.0, im = 0.0;
    if (gid < a.n) {
        cpx<T> x[12], y[12];
        SpinorIO<SP>::load(a.v[0][h], gid, x);
        SpinorIO<SP>::load(a.v[1][h], gid, y);
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            re += (double)x[k].re * y[k].re + (double)x[k].im * y[k].im;
            im += (double)x[k].re * y[k].im - (double)x[k].im * y[k].re;
        }
    }
    __shared__ double lds[256];
    const long blk = (long)blockIdx.y * gridDim.x + blockIdx.x;
    block_sum_rhs(re, gid, a.nrhs, lds, a.partials + blk, a.part_stride);
    block_sum_rhs(im, gid, a.nrhs, lds, a.partials + (long)a.nrhs * a.part_stride + blk, a.part_stride);
}

template <int SP>
__global__ void __launch_bounds__(256) k_norm2(const VecArgs a) {
    using T = typename SpinorIO<SP>::real;
    WL_FLAG_EXIT
    const int h = blockIdx.y;
    const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
    double nrm = 0.0;
    if (gid < a.n) {
        cpx<T> x[12];
        SpinorIO<SP>::load(a.v[0][h], gid, x);
#pragma unroll
        for (int k = 0; k < 12; ++k) nrm += (double)x[k].re * x[k].re + (double)x[k].im * x[k].im;
    }
    __shared__ double lds[256];
    block_sum_rhs(nrm, gid, a.nrhs, lds, a.partials + (long)blockIdx.y * gridDim.x + blockIdx.x,
                  a.part_stride);
}

template <int SP>
__global__ void __launch_bounds__(256) k_zero(const VecArgs a) {
    using T = typename SpinorIO<SP>::real;
    WL_FLAG_EXIT
    const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid < a.n) {
        cpx<T> z[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) z[k] = {T(0), T(0)};
        SpinorIO<SP>::store(a.v[0][blockIdx.y], gid, z);
    }
}

// x (FP64) += alpha p ; r -= alpha s ; partial ||r||^2
template <int SP>
__global__ void __launch_bounds__(256) k_cg_xr(const VecArgs a) {
    using T = typename SpinorIO<SP>::real;
    WL_FLAG_EXIT
    const int h = blockIdx.y;
    const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
    double nrm = 0.0;
    if (gid < a.n) {
        const int rhs = (int)(gid % a.nrhs);
        const CGScalars &sc = a.sc[rhs];
        if (sc.active) {
            const double alpha = sc.alpha;
            cpx<T> p[12], r[12], s[12];
            cpx<double> x[12];
            SpinorIO<SP>::load(a.v[1][h], gid, p);
            SpinorIO<WL_F64>::load(a.v[0][h], gid, x);
#pragma unroll
            for (int k = 0; k < 12; ++k)
                x[k] = {fma(alpha, (double)p[k].re, x[k].re), fma(alpha, (double)p[k].im, x[k].im)};
            SpinorIO<WL_F64>::store(a.v[0][h], gid, x);
            SpinorIO<SP>::load(a.v[2][h], gid, r);
            SpinorIO<SP>::load(a.v[3][h], gid, s);
            const T al = (T)alpha;
#pragma unroll
            for (int k = 0; k < 12; ++k) r[k] = {fma(-al, s[k].re, r[k].re), fma(-al, s[k].im, r[k].im)};
            SpinorIO<SP>::store(a.v[2][h], gid, r);
            if constexpr (SP != WL_F64) SpinorIO<SP>::load(a.v[2][h], gid, r);
#pragma unroll
            for (int k = 0; k < 12; ++k) nrm += (double)r[k].re * r[k].re + (double)r[k].im * r[k].im;
        }
    }
    __shared__ double lds[256];
    block_sum_rhs(nrm, gid, a.nrhs, lds, a.partials + (long)blockIdx.y * gridDim.x + blockIdx.x,
                  a.part_stride);
}

// p = r + beta p
template <int SP>
__global__ void __launch_bounds__(256) k_cg_p(const VecArgs a) {
    using T = typename SpinorIO<SP>::real;
    WL_FLAG_EXIT
    const int h = blockIdx.y;
    const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid < a.n) {
        const int rhs = (int)(gid % a.nrhs);
        if (!a.sc[rhs].active) return;
        const T beta = (T)a.sc[rhs].beta;
        cpx<T> r[12], p[12];
        SpinorIO<SP>::load(a.v[0][h], gid, r);
        SpinorIO<SP>::load(a.v[1][h], gid, p);
#pragma unroll
        for (int k = 0; k < 12; ++k) p[k] = {fma(beta, p[k].re, r[k].re), fma(beta, p[k].im, r[k].im)};
        SpinorIO<SP>::store(a.v[1][h], gid, p);
    }
}

// The rest of an iteration whose residual was updated in the hopping epilogue:
// x += alpha p (where this iteration took a step: alpha != 0, which also covers a
// system that stopped at its beta step), then p = r + beta p (systems still
// iterating).  v0 = x, v1 = p, v2 = r.  x is the FP64 solution (XP = FP64) or, in
// mixed precision, an FP32 accumulator of the steps since the last FP64 refresh
// (XP = FP32), which the solver adds to the FP64 solution before reading it.
// Launched without the active-count gate (the count is already 0 after the last
// system's final step).
template <int SP, int XP>
__global__ void __launch_bounds__(256) k_cg_xp(const VecArgs a) {
    using T = typename SpinorIO<SP>::real;
    using TX = typename SpinorIO<XP>::real;
    WL_FLAG_EXIT
    const int h = blockIdx.y;
    const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= a.n) return;
    const CGScalars &sc = a.sc[(int)(gid % a.nrhs)];
    const double alpha = sc.alpha;
    if (alpha == 0.0) return;
    cpx<T> p[12];
    SpinorIO<SP>::load(a.v[1][h], gid, p);
    cpx<TX> x[12];
    SpinorIO<XP>::load(a.v[0][h], gid, x);
    const TX ax = (TX)alpha;
#pragma unroll
    for (int k = 0; k < 12; ++k) x[k] = {fma(ax, (TX)p[k].re, x[k].re), fma(ax, (TX)p[k].im, x[k].im)};
    SpinorIO<XP>::store(a.v[0][h], gid, x);
    if (!sc.active) return;
    const T beta = (T)sc.beta;
    cpx<T> r[12];
    SpinorIO<SP>::load(a.v[2][h], gid, r);
#pragma unroll
    for (int k = 0; k < 12; ++k) p[k] = {fma(beta, p[k].re, r[k].re), fma(beta, p[k].im, r[k].im)};
    SpinorIO<SP>::store(a.v[1][h], gid, p);
}

template <int DP, int SP, bool ACC>
__global__ void __launch_bounds__(256) k_convert(const VecArgs a) {
    using TS = typename SpinorIO<SP>::real;
    using TD = typename SpinorIO<DP>::real;
    WL_FLAG_EXIT
    const int h = blockIdx.y;
    const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid < a.n) {
        cpx<TS> x[12];
        cpx<TD> y[12];
        SpinorIO<SP>::load(a.v[0][h], gid, x);
        if constexpr (ACC) {
            SpinorIO<DP>::load(a.v[1][h], gid, y);
#pragma unroll
            for (int k = 0; k < 12; ++k) y[k] = {y[k].re + (TD)x[k].re, y[k].im + (TD)x[k].im};
        } else {
#pragma unroll
            for (int k = 0; k < 12; ++k) y[k] = {(TD)x[k].re, (TD)x[k].im};
        }
        SpinorIO<DP>::store(a.v[1][h], gid, y);
    }
}

// y += (a + i b) x  (complex scalar, real a/b in the args)
template <int SP>
__global__ void __launch_bounds__(256) k_caxpy(const VecArgs a) {
    using T = typename SpinorIO<SP>::real;
    WL_FLAG_EXIT
    const int h = blockIdx.y;
    const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid < a.n) {
        cpx<T> x[12], y[12];
        SpinorIO<SP>::load(a.v[0][h], gid, x);
        SpinorIO<SP>::load(a.v[1][h], gid, y);
        const cpx<T> s = {(T)a.a, (T)a.b};
#pragma unroll
        for (int k = 0; k < 12; ++k) y[k] = cfma(s, x[k], y[k]);
        SpinorIO<SP>::store(a.v[1][h], gid, y);
    }
}

// v1 = a (1 + i b gamma_5) v0 (gamma_5 = +1 on spins 0, 1 and -1 on spins 2, 3)
template <int SP>
__global__ void __launch_bounds__(256) k_twist(const VecArgs a) {
    using T = typename SpinorIO<SP>::real;
    WL_FLAG_EXIT
    const int h = blockIdx.y;
    const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid < a.n) {
        cpx<T> x[12];
        SpinorIO<SP>::load(a.v[0][h], gid, x);
        const T sc = (T)a.a;
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            const T m = k < 6 ? (T)a.b : -(T)a.b;
            x[k] = {sc * (x[k].re - m * x[k].im), sc * (x[k].im + m * x[k].re)};
        }
        SpinorIO<SP>::store(a.v[1][h], gid, x);
    }
}

__global__ void __launch_bounds__(256) k_lincomb(const LinCombArgs a) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= a.n) return;
    double2 acc[LC_MAX_OUT];
#pragma unroll
    for (int o = 0; o < LC_MAX_OUT; ++o) acc[o] = (a.accumulate && o < a.nout) ? a.out[o][e] : make_double2(0.0, 0.0);
    for (int j = 0; j < a.nin; ++j) {
        const double2 v = a.in[j][e];
        const double2 *c = a.coef + (long)j * a.nout;
#pragma unroll
        for (int o = 0; o < LC_MAX_OUT; ++o)
            if (o < a.nout) {
                const double2 w = c[o];
                acc[o].x = fma(w.x, v.x, fma(-w.y, v.y, acc[o].x));
                acc[o].y = fma(w.x, v.y, fma(w.y, v.x, acc[o].y));
            }
    }
#pragma unroll
    for (int o = 0; o < LC_MAX_OUT; ++o)
        if (o < a.nout) a.out[o][e] = acc[o];
}

__global__ void __launch_bounds__(256) k_scale_by_rho(const VecArgs a) {
    WL_FLAG_EXIT
    const int h = blockIdx.y;
    const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= a.n) return;
    const double f = 1.0 / sqrt(a.sc[0].rho);
    cpx<double> x[12];
    SpinorIO<WL_F64>::load(a.v[0][h], gid, x);
#pragma unroll
    for (int k = 0; k < 12; ++k) x[k] = {f * x[k].re, f * x[k].im};
    SpinorIO<WL_F64>::store(a.v[1][h], gid, x);
}

__global__ void k_cg_record(const CGScalars *sc, double *hist, int cap, int *recorded) {
    if (threadIdx.x != 0) return;
    const int it = sc[0].iter;
    if (it > *recorded) {
        const int slot = (it - 1) % cap;
        hist[2 * slot] = sc[0].alpha;
        hist[2 * slot + 1] = sc[0].beta;
        *recorded = it;
    }
}

typedef double wl_d4 __attribute__((ext_vector_type(4)));

// v_mfma_f64_16x16x4f64 operands: lane l gives A[l % 16][l / 16] and B[l / 16][l % 16];
// it holds D[l / 16 + 4 i][l % 16] in component i.  The k index of a slice maps to
// element 4 (l / 16) + t of the 16-element slice in MFMA t (the same map for A and B).
__global__ void __launch_bounds__(256) k_blockdot(const BlockDotArgs a) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int q = lane >> 4, r = lane & 15;
    const double2 *wp = r < a.nw ? a.w[r] : nullptr;
    const double2 *up[4];
#pragma unroll
    for (int jt = 0; jt < 4; ++jt) up[jt] = 16 * jt + r < a.nin ? a.in[16 * jt + r] : nullptr;
    const int ntile = (a.nin + 15) >> 4;
    wl_d4 are[4], aim[4];
#pragma unroll
    for (int jt = 0; jt < 4; ++jt) are[jt] = aim[jt] = wl_d4{0.0, 0.0, 0.0, 0.0};
    const long nchunk = (a.n + 15) >> 4;
    const long nwaves = (long)gridDim.x * 4;
    for (long c = (long)blockIdx.x * 4 + wid; c < nchunk; c += nwaves) {
        const long e0 = c * 16 + 4 * q;
        double2 wv[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) wv[t] = (wp && e0 + t < a.n) ? wp[e0 + t] : make_double2(0.0, 0.0);
#pragma unroll
        for (int jt = 0; jt < 4; ++jt) {
            if (jt >= ntile) break;
            double2 uv[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) uv[t] = (up[jt] && e0 + t < a.n) ? up[jt][e0 + t] : make_double2(0.0, 0.0);
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                are[jt] = __builtin_amdgcn_mfma_f64_16x16x4f64(uv[t].x, wv[t].x, are[jt], 0, 0, 0);
                are[jt] = __builtin_amdgcn_mfma_f64_16x16x4f64(uv[t].y, wv[t].y, are[jt], 0, 0, 0);
                aim[jt] = __builtin_amdgcn_mfma_f64_16x16x4f64(uv[t].x, wv[t].y, aim[jt], 0, 0, 0);
                aim[jt] = __builtin_amdgcn_mfma_f64_16x16x4f64(-uv[t].y, wv[t].x, aim[jt], 0, 0, 0);
            }
        }
    }
    // sum the four waves: red[wave][j][o][re/im]
    __shared__ double red[4 * BD_MAX_IN * BD_MAX_W * 2];
#pragma unroll
    for (int jt = 0; jt < 4; ++jt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int j = 16 * jt + q + 4 * i;
            double *dst = red + (((size_t)wid * BD_MAX_IN + j) * BD_MAX_W + r) * 2;
            dst[0] = are[jt][i];
            dst[1] = aim[jt][i];
        }
    __syncthreads();
    const int nval = 2 * a.nin * a.nw;
    for (int v = threadIdx.x; v < nval; v += blockDim.x) {
        const int c = v & 1, jo = v >> 1, j = jo / a.nw, o = jo % a.nw;
        const size_t base = ((size_t)j * BD_MAX_W + o) * 2 + c, ws = (size_t)BD_MAX_IN * BD_MAX_W * 2;
        a.partials[(long)v * a.stride + blockIdx.x] = ((red[base] + red[base + ws]) + red[base + 2 * ws]) + red[base + 3 * ws];
    }
}

// r = b - v, partial ||r||^2
template <int SP>
__global__ void __launch_bounds__(256) k_residual(const VecArgs a) {
    using T = typename SpinorIO<SP>::real;
    WL_FLAG_EXIT
    const int h = blockIdx.y;
    const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
    double nrm = 0.0;
    if (gid < a.n) {
        cpx<T> b[12], v[12];
        SpinorIO<SP>::load(a.v[0][h], gid, b);
        SpinorIO<SP>::load(a.v[1][h], gid, v);
#pragma unroll
        for (int k = 0; k < 12; ++k) v[k] = b[k] - v[k];
        SpinorIO<SP>::store(a.v[2][h], gid, v);
        if constexpr (SP != WL_F64) SpinorIO<SP>::load(a.v[2][h], gid, v);
#pragma unroll
        for (int k = 0; k < 12; ++k) nrm += (double)v[k].re * v[k].re + (double)v[k].im * v[k].im;
    }
    __shared__ double lds[256];
    block_sum_rhs(nrm, gid, a.nrhs, lds, a.partials + (long)blockIdx.y * gridDim.x + blockIdx.x,
                  a.part_stride);
}

// ------------------------------------------------------------------ single-block reductions
// Single-block reductions of per-block partial sums run with RED_THREADS threads: each
// thread keeps four independent sums (its loads are in flight together instead of one
// dependent chain), combined in a fixed order, then the block sum; bitwise reproducible.
constexpr int RED_THREADS = 1024;

__device__ double sum_partials(const double *p, long nblk, double *lds) {
    const long st = blockDim.x;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    long b = threadIdx.x;
    for (; b + 3 * st < nblk; b += 4 * st) {
        s0 += p[b];
        s1 += p[b + st];
        s2 += p[b + 2 * st];
        s3 += p[b + 3 * st];
    }
    for (; b < nblk; b += st) s0 += p[b];
    return block_sum((s0 + s1) + (s2 + s3), lds);  // valid in thread 0
}

__global__ void __launch_bounds__(RED_THREADS) k_reduce(const double *partials, long stride, long nblk, int nvals,
                                                double *out) {
    __shared__ double lds[16];
    for (int r = 0; r < nvals; ++r) {
        const double s = sum_partials(partials + (long)r * stride, nblk, lds);
        if (threadIdx.x == 0) out[r] = s;
    }
}

__global__ void __launch_bounds__(RED_THREADS) k_reduce_rows(const double *partials, long stride, long nblk, double *out) {
    __shared__ double lds[16];
    const double s = sum_partials(partials + (long)blockIdx.x * stride, nblk, lds);
    if (threadIdx.x == 0) out[blockIdx.x] = s;
}

// One block per right-hand side.  `count` holds the number of right-hand
// sides still iterating; a system leaves the count when it stops.
__global__ void __launch_bounds__(RED_THREADS) k_cg_alpha(CGScalars *sc, const double *partials, long stride, long nblk,
                                                  const int *count) {
    // alpha = 0 marks an iteration that takes no step (read by the x update that
    // follows a fused residual update, which must run after the last system stops)
    if (count && *count == 0) {
        if (threadIdx.x == 0) sc[blockIdx.x].alpha = 0.0;
        return;
    }
    __shared__ double lds[16];
    const int r = blockIdx.x;
    CGScalars &c = sc[r];
    if (!c.active) {
        if (threadIdx.x == 0) c.alpha = 0.0;
        return;
    }
    const double s = sum_partials(partials + (long)r * stride, nblk, lds);
    if (threadIdx.x == 0) {
        c.pap = s;
        if (!(s > 0.0) || !isfinite(s) || !isfinite(c.rho)) {
            c.status = WL_BREAKDOWN;
            c.active = 0;
            c.alpha = 0.0;
            // leaves the count at the beta step of this iteration
            c.leaving = 1;
        } else {
            c.alpha = c.rho / s;
        }
    }
}

__global__ void __launch_bounds__(RED_THREADS) k_cg_beta(CGScalars *sc, const double *partials, long stride, long nblk,
                                                 int *count, int mode) {
    if (*count == 0) return;
    __shared__ double lds[16];
    const int r = blockIdx.x;
    CGScalars &c = sc[r];
    if (!c.active) {
        if (threadIdx.x == 0) {
            c.beta = 0.0;
            if (c.leaving) {
                c.leaving = 0;
                atomicSub(count, 1);
            }
        }
        return;
    }
    const double s = sum_partials(partials + (long)r * stride, nblk, lds);
    if (threadIdx.x == 0) {
        c.beta = 0.0;
        c.iter += 1;
        if (!isfinite(s)) {
            c.status = WL_BREAKDOWN;
            c.active = 0;
        } else {
            // mode 0: plain step; 1: the residual was just refreshed in FP64 (restart
            // the rho_max record); 2: also restart the search direction.  In mode 1 a
            // refresh that finds the true residual more than twice the iterated one
            // (the iterated residual had drifted far below it) restarts the direction
            // as well: the old direction then says nothing about the new residual, and
            // beta = rho'/rho would be large and let it dominate.
            const bool restart = mode == 2 || (mode == 1 && s > 4.0 * c.rho_iter);
            c.beta = restart ? 0.0 : s / c.rho;
            c.rho = s;
            c.rho_max = mode ? s : fmax(c.rho_max, s);
            if (s <= c.target) {
                c.status = WL_OK;
                c.active = 0;
            } else if (c.iter >= c.maxiter) {
                c.status = WL_NOT_CONVERGED;
                c.active = 0;
            }
        }
        if (!c.active) atomicSub(count, 1);
    }
}

__global__ void __launch_bounds__(RED_THREADS) k_cg_stash(CGScalars *sc, const double *partials, long stride, long nblk,
                                                  const int *count) {
    if (count && *count == 0) return;
    __shared__ double lds[16];
    const int r = blockIdx.x;
    CGScalars &c = sc[r];
    if (!c.active) return;
    const double s = sum_partials(partials + (long)r * stride, nblk, lds);
    if (threadIdx.x == 0) c.rho_iter = s;
}

__global__ void __launch_bounds__(RED_THREADS) k_cg_init(CGScalars *sc, int nrhs, const double *partials, long stride,
                                                 long nblk, const double *bnorm2, double tol, int maxiter,
                                                 int *count) {
    __shared__ double lds[16];
    int any = 0;
    for (int r = 0; r < nrhs; ++r) {
        const double s = sum_partials(partials + (long)r * stride, nblk, lds);
        if (threadIdx.x == 0) {
            CGScalars &c = sc[r];
            c.rho = s;
            c.rho_max = s;
            c.pap = 0.0;
            c.alpha = 0.0;
            c.beta = 0.0;
            c.target = tol * tol * bnorm2[r];
            c.iter = 0;
            c.maxiter = maxiter;
            c.leaving = 0;
            c.rho_iter = s;
            if (!isfinite(s)) {
                c.status = WL_BREAKDOWN;
                c.active = 0;
            } else if (s <= c.target) {
                c.status = WL_OK;
                c.active = 0;
            } else if (maxiter <= 0) {
                c.status = WL_NOT_CONVERGED;
                c.active = 0;
            } else {
                c.status = WL_NOT_CONVERGED;
                c.active = 1;
            }
            any += c.active;
        }
    }
    if (threadIdx.x == 0) *count = any;
}

// ------------------------------------------------------------------ launchers
#define WL_DISPATCH_PREC(prec, KERNEL, ...)                                                            \
    switch (prec) {                                                                                    \
    case WL_F64: hipLaunchKernelGGL((KERNEL<WL_F64 __VA_ARGS__>), grid, dim3(blas_block()), 0, s, a); break;   \
    case WL_F32: hipLaunchKernelGGL((KERNEL<WL_F32 __VA_ARGS__>), grid, dim3(blas_block()), 0, s, a); break;   \
    case WL_F16N: hipLaunchKernelGGL((KERNEL<WL_F16N __VA_ARGS__>), grid, dim3(blas_block()), 0, s, a); break; \
    case WL_BF16N: hipLaunchKernelGGL((KERNEL<WL_BF16N __VA_ARGS__>), grid, dim3(blas_block()), 0, s, a); break; \
    case WL_I16N: hipLaunchKernelGGL((KERNEL<WL_I16N __VA_ARGS__>), grid, dim3(blas_block()), 0, s, a); break; \
    default: return hipErrorInvalidValue;                                                              \
    }                                                                                                  \
    return hipGetLastError();

static dim3 vgrid(const VecArgs &a, int nh) { return dim3((unsigned)blas_blocks(a.n), (unsigned)nh); }

hipError_t blas_axpby(int prec, VecArgs &a, int nh, bool norm, hipStream_t s) {
    dim3 grid = vgrid(a, nh);
    if (norm) {
        WL_DISPATCH_PREC(prec, k_axpby, , true)
    } else {
        WL_DISPATCH_PREC(prec, k_axpby, , false)
    }
}
hipError_t blas_lincomb(const LinCombArgs &a, hipStream_t s) {
    if (a.nin < 1 || a.nin > LC_MAX_IN || a.nout < 1 || a.nout > LC_MAX_OUT || a.n < 0) return hipErrorInvalidValue;
    if (a.n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_lincomb, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}
long blockdot_blocks(long n) { return std::max(1L, std::min(512L, ((n + 15) / 16 + 3) / 4)); }
hipError_t blas_blockdot(const BlockDotArgs &a, hipStream_t s) {
    if (a.nin < 1 || a.nin > BD_MAX_IN || a.nw < 1 || a.nw > BD_MAX_W || a.n < 0 || !a.partials ||
        a.stride < blockdot_blocks(a.n))
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_blockdot, dim3((unsigned)blockdot_blocks(a.n)), dim3(256), 0, s, a);
    return hipGetLastError();
}
hipError_t cg_update_xp(int prec, int xprec, VecArgs &a, int nh, hipStream_t s) {
    dim3 grid = vgrid(a, nh);
    if (xprec == WL_F32) {
        WL_DISPATCH_PREC(prec, k_cg_xp, , WL_F32)
    }
    if (xprec != WL_F64) return hipErrorInvalidValue;
    WL_DISPATCH_PREC(prec, k_cg_xp, , WL_F64)
}
hipError_t blas_scale_by_rho(VecArgs &a, int nh, hipStream_t s) {
    if (!a.sc || a.nrhs != 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_scale_by_rho, vgrid(a, nh), dim3(blas_block()), 0, s, a);
    return hipGetLastError();
}
hipError_t cg_record(const CGScalars *sc, double *hist, int cap, int *recorded, hipStream_t s) {
    if (cap < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_cg_record, dim3(1), dim3(64), 0, s, sc, hist, cap, recorded);
    return hipGetLastError();
}
hipError_t reduce_rows(const double *partials, long stride, long nblk, int nvals, double *out, hipStream_t s) {
    if (nvals < 1 || nblk < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_reduce_rows, dim3((unsigned)nvals), dim3(RED_THREADS), 0, s, partials, stride, nblk, out);
    return hipGetLastError();
}
hipError_t blas_twist(int prec, VecArgs &a, int nh, hipStream_t s) {
    dim3 grid = vgrid(a, nh);
    WL_DISPATCH_PREC(prec, k_twist)
}
hipError_t blas_dot(int prec, VecArgs &a, int nh, hipStream_t s) {
    dim3 grid = vgrid(a, nh);
    WL_DISPATCH_PREC(prec, k_dot)
}
hipError_t blas_norm2(int prec, VecArgs &a, int nh, hipStream_t s) {
    dim3 grid = vgrid(a, nh);
    WL_DISPATCH_PREC(prec, k_norm2)
}
hipError_t blas_zero(int prec, VecArgs &a, int nh, hipStream_t s) {
    dim3 grid = vgrid(a, nh);
    WL_DISPATCH_PREC(prec, k_zero)
}
hipError_t cg_update_xr(int prec, int xprec, VecArgs &a, int nh, hipStream_t s) {
    if (xprec != WL_F64) return hipErrorInvalidValue;
    dim3 grid = vgrid(a, nh);
    WL_DISPATCH_PREC(prec, k_cg_xr)
}
hipError_t cg_update_p(int prec, VecArgs &a, int nh, hipStream_t s) {
    dim3 grid = vgrid(a, nh);
    WL_DISPATCH_PREC(prec, k_cg_p)
}
hipError_t blas_caxpy(int prec, VecArgs &a, int nh, hipStream_t s) {
    dim3 grid = vgrid(a, nh);
    WL_DISPATCH_PREC(prec, k_caxpy)
}
hipError_t blas_residual(int prec, VecArgs &a, int nh, hipStream_t s) {
    dim3 grid = vgrid(a, nh);
    WL_DISPATCH_PREC(prec, k_residual)
}

template <int DP, bool ACC>
static hipError_t convert_src(int sprec, VecArgs &a, dim3 grid, hipStream_t s) {
    switch (sprec) {
    case WL_F64: hipLaunchKernelGGL((k_convert<DP, WL_F64, ACC>), grid, dim3(blas_block()), 0, s, a); break;
    case WL_F32: hipLaunchKernelGGL((k_convert<DP, WL_F32, ACC>), grid, dim3(blas_block()), 0, s, a); break;
    case WL_F16N: hipLaunchKernelGGL((k_convert<DP, WL_F16N, ACC>), grid, dim3(blas_block()), 0, s, a); break;
    case WL_BF16N: hipLaunchKernelGGL((k_convert<DP, WL_BF16N, ACC>), grid, dim3(blas_block()), 0, s, a); break;
    case WL_I16N: hipLaunchKernelGGL((k_convert<DP, WL_I16N, ACC>), grid, dim3(blas_block()), 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
template <bool ACC>
static hipError_t convert_dst(int dprec, int sprec, VecArgs &a, dim3 grid, hipStream_t s) {
    switch (dprec) {
    case WL_F64: return convert_src<WL_F64, ACC>(sprec, a, grid, s);
    case WL_F32: return convert_src<WL_F32, ACC>(sprec, a, grid, s);
    case WL_F16N: return convert_src<WL_F16N, ACC>(sprec, a, grid, s);
    case WL_BF16N: return convert_src<WL_BF16N, ACC>(sprec, a, grid, s);
    case WL_I16N: return convert_src<WL_I16N, ACC>(sprec, a, grid, s);
    default: return hipErrorInvalidValue;
    }
}
hipError_t blas_convert(int dprec, int sprec, bool acc, VecArgs &a, int nh, hipStream_t s) {
    dim3 grid = vgrid(a, nh);
    return acc ? convert_dst<true>(dprec, sprec, a, grid, s) : convert_dst<false>(dprec, sprec, a, grid, s);
}

hipError_t reduce_partials(const double *partials, long stride, long nblk, int nvals, double *out,
                           hipStream_t s) {
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(RED_THREADS), 0, s, partials, stride, nblk, nvals, out);
    return hipGetLastError();
}
hipError_t cg_alpha(CGScalars *sc, int nrhs, const double *partials, long stride, long nblk,
                    const int *flag, hipStream_t s) {
    hipLaunchKernelGGL(k_cg_alpha, dim3(nrhs), dim3(RED_THREADS), 0, s, sc, partials, stride, nblk, flag);
    return hipGetLastError();
}
hipError_t cg_beta(CGScalars *sc, int nrhs, const double *partials, long stride, long nblk, int *done,
                   int mode, hipStream_t s) {
    hipLaunchKernelGGL(k_cg_beta, dim3(nrhs), dim3(RED_THREADS), 0, s, sc, partials, stride, nblk, done, mode);
    return hipGetLastError();
}
hipError_t cg_stash_rho(CGScalars *sc, int nrhs, const double *partials, long stride, long nblk, const int *flag,
                        hipStream_t s) {
    hipLaunchKernelGGL(k_cg_stash, dim3(nrhs), dim3(RED_THREADS), 0, s, sc, partials, stride, nblk, flag);
    return hipGetLastError();
}
hipError_t cg_init(CGScalars *sc, int nrhs, const double *partials, long stride, long nblk,
                   const double *bnorm2, double tol, int maxiter, int *done, hipStream_t s) {
    hipLaunchKernelGGL(k_cg_init, dim3(1), dim3(RED_THREADS), 0, s, sc, nrhs, partials, stride, nblk, bnorm2, tol,
                       maxiter, done);
    return hipGetLastError();
}

// ------------------------------------------------------------------ inner CG of the preconditioned normal equations
__global__ void __launch_bounds__(RED_THREADS) k_pcg_start(PcgScalars *sc, const double *partials, long stride,
                                                            long nblk, const double *rho2_start, const double *stop2,
                                                            const int *live, int *count) {
    __shared__ double lds[16];
    const int r = blockIdx.x;
    const double g = sum_partials(partials + (long)r * stride, nblk, lds);
    if (threadIdx.x == 0) {
        PcgScalars &c = sc[r];
        c.gam = g;
        c.alpha = 0.0;
        c.beta = 0.0;
        c.rho2 = rho2_start[r];
        c.stop2 = stop2[r];
        c.iters = 0;
        c.breakdown = 0;
        c.active = live[r] && c.rho2 > c.stop2 ? 1 : 0;
        if (c.active && (!(g > 0.0) || !isfinite(g))) {
            c.active = 0;
            c.breakdown = 1;
        }
        if (c.active) atomicAdd(count, 1);
    }
}

__global__ void __launch_bounds__(RED_THREADS) k_pcg_alpha(PcgScalars *sc, const double *partials, long stride,
                                                            long nblk, int *count) {
    __shared__ double lds[16];
    const int r = blockIdx.x;
    PcgScalars &c = sc[r];
    if (!c.active) {
        if (threadIdx.x == 0) c.alpha = 0.0;
        return;
    }
    const double q2 = sum_partials(partials + (long)r * stride, nblk, lds);
    if (threadIdx.x == 0) {
        if (!(q2 > 0.0) || !isfinite(q2)) {
            c.alpha = 0.0;
            c.active = 0;
            c.breakdown = 1;
            atomicSub(count, 1);
        } else {
            c.alpha = c.gam / q2;
        }
    }
}

__global__ void __launch_bounds__(256) k_pcg_update_yr(const PcgVec v) {
    const int h = blockIdx.y;
    const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
    double nrm = 0.0;
    if (gid < v.n) {
        const int rhs = (int)(gid % v.nrhs);
        const double alpha = v.sc[rhs].alpha;
        cpx<float> r[12];
        SpinorIO<WL_F32>::load(v.rho[h], gid, r);
        if (alpha != 0.0) {
            cpx<float> y[12], p[12], q[12];
            SpinorIO<WL_F32>::load(v.y[h], gid, y);
            SpinorIO<WL_F32>::load(v.p[h], gid, p);
            SpinorIO<WL_F32>::load(v.q[h], gid, q);
            const float al = (float)alpha;
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                y[k] = {fmaf(al, p[k].re, y[k].re), fmaf(al, p[k].im, y[k].im)};
                r[k] = {fmaf(-al, q[k].re, r[k].re), fmaf(-al, q[k].im, r[k].im)};
            }
            SpinorIO<WL_F32>::store(v.y[h], gid, y);
            SpinorIO<WL_F32>::store(v.rho[h], gid, r);
        }
#pragma unroll
        for (int k = 0; k < 12; ++k) nrm += (double)r[k].re * r[k].re + (double)r[k].im * r[k].im;
    }
    __shared__ double lds[256];
    block_sum_rhs(nrm, gid, v.nrhs, lds, v.partials + (long)blockIdx.y * gridDim.x + blockIdx.x, v.part_stride);
}

__global__ void __launch_bounds__(RED_THREADS) k_pcg_check(PcgScalars *sc, const double *partials, long stride,
                                                            long nblk, int *count) {
    __shared__ double lds[16];
    const int r = blockIdx.x;
    PcgScalars &c = sc[r];
    if (!c.active) return;
    const double s2 = sum_partials(partials + (long)r * stride, nblk, lds);
    if (threadIdx.x == 0) {
        c.rho2 = s2;
        c.iters += 1;
        if (!isfinite(s2)) c.breakdown = 1;
        if (!isfinite(s2) || s2 <= c.stop2) {
            c.active = 0;
            atomicSub(count, 1);
        }
    }
}

__global__ void __launch_bounds__(RED_THREADS) k_pcg_beta(PcgScalars *sc, const double *partials, long stride,
                                                           long nblk, int *count) {
    __shared__ double lds[16];
    const int r = blockIdx.x;
    PcgScalars &c = sc[r];
    if (!c.active) return;
    const double g1 = sum_partials(partials + (long)r * stride, nblk, lds);
    if (threadIdx.x == 0) {
        if (!isfinite(g1)) {
            c.beta = 0.0;
            c.active = 0;
            c.breakdown = 1;
            atomicSub(count, 1);
        } else {
            c.beta = g1 / c.gam;
            c.gam = g1;
        }
    }
}

__global__ void __launch_bounds__(256) k_pcg_update_p(const PcgVec v) {
    const int h = blockIdx.y;
    const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= v.n) return;
    const PcgScalars &c = v.sc[(int)(gid % v.nrhs)];
    if (!c.active) return;
    const float beta = (float)c.beta;
    cpx<float> sv[12], p[12];
    SpinorIO<WL_F32>::load(v.q[h], gid, sv);
    SpinorIO<WL_F32>::load(v.p[h], gid, p);
#pragma unroll
    for (int k = 0; k < 12; ++k) p[k] = {fmaf(beta, p[k].re, sv[k].re), fmaf(beta, p[k].im, sv[k].im)};
    SpinorIO<WL_F32>::store(v.p[h], gid, p);
}

hipError_t pcg_start(PcgScalars *sc, int nrhs, const double *partials, long stride, long nblk,
                     const double *rho2_start, const double *stop2, const int *live, int *count, hipStream_t s) {
    hipLaunchKernelGGL(k_pcg_start, dim3(nrhs), dim3(RED_THREADS), 0, s, sc, partials, stride, nblk, rho2_start,
                       stop2, live, count);
    return hipGetLastError();
}
hipError_t pcg_alpha(PcgScalars *sc, int nrhs, const double *partials, long stride, long nblk, int *count,
                     hipStream_t s) {
    hipLaunchKernelGGL(k_pcg_alpha, dim3(nrhs), dim3(RED_THREADS), 0, s, sc, partials, stride, nblk, count);
    return hipGetLastError();
}
hipError_t pcg_update_yr(const PcgVec &v, hipStream_t s) {
    hipLaunchKernelGGL(k_pcg_update_yr, dim3((unsigned)blas_blocks(v.n), 2), dim3(256), 0, s, v);
    return hipGetLastError();
}
hipError_t pcg_check(PcgScalars *sc, int nrhs, const double *partials, long stride, long nblk, int *count,
                     hipStream_t s) {
    hipLaunchKernelGGL(k_pcg_check, dim3(nrhs), dim3(RED_THREADS), 0, s, sc, partials, stride, nblk, count);
    return hipGetLastError();
}
hipError_t pcg_beta(PcgScalars *sc, int nrhs, const double *partials, long stride, long nblk, int *count,
                    hipStream_t s) {
    hipLaunchKernelGGL(k_pcg_beta, dim3(nrhs), dim3(RED_THREADS), 0, s, sc, partials, stride, nblk, count);
    return hipGetLastError();
}
hipError_t pcg_update_p(const PcgVec &v, hipStream_t s) {
    hipLaunchKernelGGL(k_pcg_update_p, dim3((unsigned)blas_blocks(v.n), 2), dim3(256), 0, s, v);
    return hipGetLastError();
}

template <int SP>
__global__ void __launch_bounds__(256) k_zero_masked(char *f, size_t half, long n, int nrhs, const int *mask) {
    using T = typename SpinorIO<SP>::real;
    const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= n || !mask[gid % nrhs]) return;
    cpx<T> z[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) z[k] = {T(0), T(0)};
    SpinorIO<SP>::store(f + blockIdx.y * half, gid, z);
}

hipError_t blas_zero_masked(int prec, void *f, size_t half, long n, int nrhs, const int *mask, hipStream_t s) {
    dim3 grid((unsigned)blas_blocks(n), 2);
    if (prec == WL_F64) hipLaunchKernelGGL(k_zero_masked<WL_F64>, grid, dim3(256), 0, s, (char *)f, half, n, nrhs, mask);
    else if (prec == WL_F32) hipLaunchKernelGGL(k_zero_masked<WL_F32>, grid, dim3(256), 0, s, (char *)f, half, n, nrhs, mask);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace wl
