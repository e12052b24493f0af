// Device code of the hopping-term kernels (included by the translation units
// that instantiate them).
#pragma once

#include "wl_dslash.h"


namespace wl {

// -i a
template <typename T> __device__ __forceinline__ cpx<T> mi(cpx<T> a) { return {a.im, -a.re}; }

// Neighbour spinor of a hop: f = its components divided by the returned
// factor.  BF16 and int16 storage return the stored numbers and their point's
// norm (times the format's fixed scale), so that a hop applies the norm once,
// to its SU(3) product in the accumulate (multiply-adds that replace the
// additions), instead of to all 24 inputs: 4-7 % faster half-dslash.  The other
// formats return the components and 1, which folds away.  (FP16 keeps the
// scaled load: its decode already fuses into mixed-precision multiply-adds,
// and the late norm costs two registers that take a wave from its kernels.)
template <int SP>
__device__ __forceinline__ typename SpinorIO<SP>::real load_nb(const void *base, long i,
                                                               cpx<typename SpinorIO<SP>::real> f[12]) {
    if constexpr (SP == WL_BF16N || SP == WL_I16N) {
        return SpinorIO<SP>::load_unscaled(base, i, f);
    } else {
        SpinorIO<SP>::load(base, i, f);
        return 1;
    }
}

// acc + k * v, componentwise
template <typename T> __device__ __forceinline__ cpx<T> pacc(cpx<T> acc, cpx<T> v, T k) {
    return {fma(k, v.re, acc.re), fma(k, v.im, acc.im)};
}

// v[k] <- (1 + i m gamma_5) v[k] for N consecutive components starting at
// component `first` of a spinor (component 3 spin + colour; gamma_5 = +1 on
// spins 0 and 1, -1 on spins 2 and 3 in the chiral basis)
template <typename T, int N>
__device__ __forceinline__ void twist(cpx<T> *v, int first, T m) {
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const T s = first + k < 6 ? m : -m;
        v[k] = {v[k].re - s * v[k].im, v[k].im + s * v[k].re};
    }
}

// h = upper + S * A_mu * lower for both upper spin rows, colour c.
// A_x = -i s1, A_y = -i s2, A_z = -i s3, A_t = -1.
template <typename T, int MU, int S>
__device__ __forceinline__ void project(const cpx<T> f[12], cpx<T> h[6]) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const cpx<T> u0 = f[c], u1 = f[3 + c], l0 = f[6 + c], l1 = f[9 + c];
        if constexpr (MU == 0) {  // A lo = (-i l1, -i l0)
            h[c] = S > 0 ? u0 + mi(l1) : u0 - mi(l1);
            h[3 + c] = S > 0 ? u1 + mi(l0) : u1 - mi(l0);
        } else if constexpr (MU == 1) {  // A lo = (-l1, l0)
            h[c] = S > 0 ? u0 - l1 : u0 + l1;
            h[3 + c] = S > 0 ? u1 + l0 : u1 - l0;
        } else if constexpr (MU == 2) {  // A lo = (-i l0, i l1)
            h[c] = S > 0 ? u0 + mi(l0) : u0 - mi(l0);
            h[3 + c] = S > 0 ? u1 + ti(l1) : u1 - ti(l1);
        } else {  // A lo = (-l0, -l1)
            h[c] = S > 0 ? u0 - l0 : u0 + l0;
            h[3 + c] = S > 0 ? u1 - l1 : u1 + l1;
        }
    }
}

// acc_up += sc v ; acc_lo += S sc A_mu^+ v (sc: the neighbour's factor, see load_nb).
// A_x^+ v = (i v1, i v0), A_y^+ v = (v1, -v0), A_z^+ v = (i v0, -i v1), A_t^+ v = -v.
template <typename T, int MU, int S>
__device__ __forceinline__ void accumulate(cpx<T> acc[12], const cpx<T> v[6], T sc) {
    const T ssc = S > 0 ? sc : -sc;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const cpx<T> v0 = v[c], v1 = v[3 + c];
        acc[c] = pacc(acc[c], v0, sc);
        acc[3 + c] = pacc(acc[3 + c], v1, sc);
        cpx<T> w0, w1;
        if constexpr (MU == 0) {
            w0 = ti(v1);
            w1 = ti(v0);
        } else if constexpr (MU == 1) {
            w0 = v1;
            w1 = -v0;
        } else if constexpr (MU == 2) {
            w0 = ti(v0);
            w1 = mi(v1);
        } else {
            w0 = -v0;
            w1 = -v1;
        }
        acc[6 + c] = pacc(acc[6 + c], w0, ssc);
        acc[9 + c] = pacc(acc[9 + c], w1, ssc);
    }
}

// v = U h (FWD) or U^+ h (backward), both spin rows
template <typename T, bool FWD>
__device__ __forceinline__ void su3_mul2(const cpx<T> u[9], const cpx<T> h[6], cpx<T> v[6]) {
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            cpx<T> r;
            if constexpr (FWD) {
                r = cmul(u[3 * i], h[3 * s]);
                r = cfma(u[3 * i + 1], h[3 * s + 1], r);
                r = cfma(u[3 * i + 2], h[3 * s + 2], r);
            } else {
                r = cjmul(u[i], h[3 * s]);
                r = cjfma(u[3 + i], h[3 * s + 1], r);
                r = cjfma(u[6 + i], h[3 * s + 2], r);
            }
            v[3 * s + i] = r;
        }
}

// Neighbour of even/odd site i (coordinates c, xh = c[0] / 2) one hop along +-MU:
// its index j (in the other parity's field) and whether the hop wraps.
template <int MU, bool FWD>
__device__ __forceinline__ void hop_neighbour(const Geom &g, int i, int xh, const int c[4], int &j, bool &wrap) {
    if constexpr (MU == 0) {
        int x = c[0] + (FWD ? 1 : -1);
        wrap = FWD ? (x == g.L[0]) : (x < 0);
        if (wrap) x = FWD ? 0 : g.L[0] - 1;
        j = (i - xh) + (x >> 1);
    } else {
        const int stride = MU == 1 ? g.sy : (MU == 2 ? g.sz : g.st);
        wrap = FWD ? (c[MU] == g.L[MU] - 1) : (c[MU] == 0);
        j = FWD ? i + stride : i - stride;
        if (wrap) j += FWD ? -g.L[MU] * stride : g.L[MU] * stride;
    }
}

// One hop with the neighbour's spinor f given: project, multiply by the link
// (loaded here), boundary phase, accumulate.
template <int SP, int GP, int RECON, bool DAG, bool NT, int MU, bool FWD>
__device__ __forceinline__ void hop_apply(const HopArgs &a, int par, int i, int j, bool wrap,
                                          const cpx<typename SpinorIO<SP>::real> f[12],
                                          typename SpinorIO<SP>::real sc, cpx<typename SpinorIO<SP>::real> acc[12]) {
    using T = typename SpinorIO<SP>::real;
    const Geom &g = a.g;
    // Forward hop (H): (1 - gamma) -> S = -1; backward: (1 + gamma) -> S = +1; H^+ swaps them.
    constexpr int S = (FWD != DAG) ? -1 : 1;
    cpx<T> h[6], u[9], v[6];
    const int lpar = FWD ? par : 1 - par;
    const char *slab = (const char *)a.gauge + (size_t)(lpar * 4 + MU) * a.slab_bytes;
    LinkIO<GP, RECON>::template load<NT>(slab, FWD ? i : j, u);
    project<T, MU, S>(f, h);
    su3_mul2<T, FWD>(u, h, v);
    if (wrap && ((g.phase_mask >> MU) & 1)) {
        const cpx<T> z = {(T)g.zr[MU], FWD ? (T)g.zi[MU] : -(T)g.zi[MU]};
#pragma unroll
        for (int k = 0; k < 6; ++k) v[k] = cmul(z, v[k]);
    }
    accumulate<T, MU, S>(acc, v, sc);
}

template <int SP, int GP, int RECON, bool DAG, bool NT, int MU, bool FWD>
__device__ __forceinline__ void hop(const HopArgs &a, int par, int i, int xh, const int c[4], int rhs,
                                    cpx<typename SpinorIO<SP>::real> acc[12]) {
    using T = typename SpinorIO<SP>::real;
    int j;
    bool wrap;
    hop_neighbour<MU, FWD>(a.g, i, xh, c, j, wrap);
    cpx<T> f[12];
    const T sc = load_nb<SP>(a.in[1 - par], (long)j * a.nrhs + rhs, f);
    hop_apply<SP, GP, RECON, DAG, NT, MU, FWD>(a, par, i, j, wrap, f, sc, acc);
}

// The same hop for R consecutive right-hand sides of one site: the link is
// loaded (and reconstructed) once and applied to all R neighbour spinors.
template <int SP, int GP, int RECON, bool DAG, bool NT, int MU, bool FWD, int R>
__device__ __forceinline__ void hop_r(const HopArgs &a, int par, int i, int xh, const int c[4], int rhs0,
                                      cpx<typename SpinorIO<SP>::real> (&acc)[R][12]) {
    using T = typename SpinorIO<SP>::real;
    const Geom &g = a.g;
    int j;
    bool wrap;
    if constexpr (MU == 0) {
        int x = c[0] + (FWD ? 1 : -1);
        wrap = FWD ? (x == g.L[0]) : (x < 0);
        if (wrap) x = FWD ? 0 : g.L[0] - 1;
        j = (i - xh) + (x >> 1);
    } else {
        const int stride = MU == 1 ? g.sy : (MU == 2 ? g.sz : g.st);
        wrap = FWD ? (c[MU] == g.L[MU] - 1) : (c[MU] == 0);
        j = FWD ? i + stride : i - stride;
        if (wrap) j += FWD ? -g.L[MU] * stride : g.L[MU] * stride;
    }
    constexpr int S = (FWD != DAG) ? -1 : 1;
    cpx<T> u[9];
    const int lpar = FWD ? par : 1 - par;
    const char *slab = (const char *)a.gauge + (size_t)(lpar * 4 + MU) * a.slab_bytes;
    LinkIO<GP, RECON>::template load<NT>(slab, FWD ? i : j, u);
    const bool ph = wrap && ((g.phase_mask >> MU) & 1);
    const cpx<T> z = {(T)g.zr[MU], FWD ? (T)g.zi[MU] : -(T)g.zi[MU]};
#pragma unroll
    for (int r = 0; r < R; ++r) {
        cpx<T> f[12], h[6], v[6];
        const T sc = load_nb<SP>(a.in[1 - par], (long)j * a.nrhs + rhs0 + r, f);
        project<T, MU, S>(f, h);
        su3_mul2<T, FWD>(u, h, v);
        if (ph) {
#pragma unroll
            for (int k = 0; k < 6; ++k) v[k] = cmul(z, v[k]);
        }
        accumulate<T, MU, S>(acc[r], v, sc);
    }
}

// ---- split variant: the direction of the hop (forward / backward) is a
// per-lane runtime value, so that both halves of a wavefront run the same
// instruction stream; the projector sign becomes a runtime +-1 and the
// backward link is transposed and conjugated by selects.

// h = upper + s * A_mu * lower
template <typename T, int MU>
__device__ __forceinline__ void project_rt(const cpx<T> f[12], T s, cpx<T> h[6]) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const cpx<T> u0 = f[c], u1 = f[3 + c], l0 = f[6 + c], l1 = f[9 + c];
        cpx<T> a0, a1;
        if constexpr (MU == 0) {
            a0 = mi(l1);
            a1 = mi(l0);
        } else if constexpr (MU == 1) {
            a0 = -l1;
            a1 = l0;
        } else if constexpr (MU == 2) {
            a0 = mi(l0);
            a1 = ti(l1);
        } else {
            a0 = -l0;
            a1 = -l1;
        }
        h[c] = {fma(s, a0.re, u0.re), fma(s, a0.im, u0.im)};
        h[3 + c] = {fma(s, a1.re, u1.re), fma(s, a1.im, u1.im)};
    }
}

// acc_up += sc v ; acc_lo += s sc A_mu^+ v (sc: the neighbour's factor, see load_nb)
template <typename T, int MU>
__device__ __forceinline__ void accumulate_rt(cpx<T> acc[12], const cpx<T> v[6], T s, T sc) {
    const T ssc = s * sc;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const cpx<T> v0 = v[c], v1 = v[3 + c];
        acc[c] = pacc(acc[c], v0, sc);
        acc[3 + c] = pacc(acc[3 + c], v1, sc);
        cpx<T> w0, w1;
        if constexpr (MU == 0) {
            w0 = ti(v1);
            w1 = ti(v0);
        } else if constexpr (MU == 1) {
            w0 = v1;
            w1 = -v0;
        } else if constexpr (MU == 2) {
            w0 = ti(v0);
            w1 = mi(v1);
        } else {
            w0 = -v0;
            w1 = -v1;
        }
        acc[6 + c] = pacc(acc[6 + c], w0, ssc);
        acc[9 + c] = pacc(acc[9 + c], w1, ssc);
    }
}

template <int SP, int GP, int RECON, bool DAG, bool NT, int MU>
__device__ __forceinline__ void hop_rt(const HopArgs &a, int par, int i, int xh, const int c[4], int rhs, bool fwd,
                                       cpx<typename SpinorIO<SP>::real> acc[12]) {
    using T = typename SpinorIO<SP>::real;
    const Geom &g = a.g;
    int j;
    bool wrap;
    if constexpr (MU == 0) {
        int x = c[0] + (fwd ? 1 : -1);
        wrap = fwd ? (x == g.L[0]) : (x < 0);
        if (wrap) x = fwd ? 0 : g.L[0] - 1;
        j = (i - xh) + (x >> 1);
    } else {
        const int stride = MU == 1 ? g.sy : (MU == 2 ? g.sz : g.st);
        wrap = fwd ? (c[MU] == g.L[MU] - 1) : (c[MU] == 0);
        j = fwd ? i + stride : i - stride;
        if (wrap) j += fwd ? -g.L[MU] * stride : g.L[MU] * stride;
    }
    const T s = (fwd != DAG) ? T(-1) : T(1);
    cpx<T> f[12], h[6], u[9], w[9], v[6];
    const T sc = load_nb<SP>(a.in[1 - par], (long)j * a.nrhs + rhs, f);
    const int lpar = fwd ? par : 1 - par;
    const char *slab = (const char *)a.gauge + (size_t)(lpar * 4 + MU) * a.slab_bytes;
    LinkIO<GP, RECON>::template load<NT>(slab, fwd ? i : j, u);
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int q = 0; q < 3; ++q) w[3 * r + q] = fwd ? u[3 * r + q] : conjg(u[3 * q + r]);
    project_rt<T, MU>(f, s, h);
    su3_mul2<T, true>(w, h, v);
    if (wrap && ((g.phase_mask >> MU) & 1)) {
        const cpx<T> z = {(T)g.zr[MU], fwd ? (T)g.zi[MU] : -(T)g.zi[MU]};
#pragma unroll
        for (int k = 0; k < 6; ++k) v[k] = cmul(z, v[k]);
    }
    accumulate_rt<T, MU>(acc, v, s, sc);
}

// Site position and right-hand side of point gid of the processing order (rhs
// fastest).  Points of a launch stay below 2^31 (checked by the launchers), so
// the index arithmetic is 32-bit: 64-bit division is a long software sequence.
__device__ __forceinline__ int pos_of_point(const HopArgs &a, long gid, int &rhs) {
    const int g = (int)gid;
    if (a.nrhs == 1) {
        rhs = 0;
        return g;
    }
    const int ps = g / a.nrhs;
    rhs = g - ps * a.nrhs;
    return ps;
}

// e/o index of the site at position ps of the processing order
__device__ __forceinline__ int site_of(const HopArgs &a, int ps) {
    if (a.tchunk == 0) return ps;
    const Geom &g = a.g;
    if (a.tchunk == WL_TCHUNK_YZ) return yz_site(g, a.yz_by, a.yz_bz, a.f_blk, a.f_slab, a.f_row, ps);
    const int plane = g.sz;  // (Lx/2) * Ly sites of one (z, t)
    if (a.tchunk < 0) {
        // chunks of -tchunk z-planes over all t, each walked with t slowest
        const int k = -a.tchunk;
        const int chunk = fdiv(ps, a.f_chunk);
        const int r = ps - chunk * a.chunk_sites;
        const int z0 = chunk * k;
        const int kz = min(k, g.L[2] - z0);  // the last chunk may be thinner
        const int t = kz == k ? fdiv(r, a.f_kplane) : r / (kz * plane);
        const int q = r - t * kz * plane;
        const int zl = fdiv(q, g.f_sz);
        return (q - zl * plane) + plane * (z0 + zl) + g.st * t;
    }
    const int chunk = ps / a.chunk_sites;
    const int r = ps - chunk * a.chunk_sites;
    const int t0 = chunk * a.tchunk;
    const int trc = min(a.tchunk, g.L[3] - t0);  // the last chunk may be shorter
    const int yx = r % plane;
    const int q = r / plane;
    const int tl = q % trc, z = q / trc;
    return yx + plane * (z + g.L[2] * (t0 + tl));
}

__device__ __forceinline__ long logical_block(int swizzle) {
    const long nb = gridDim.x, bid = blockIdx.x;
    if (!swizzle || nb < 16) return bid;
    // hardware dispatches block b to XCD b % 8: give XCD x one contiguous range
    const long q = nb / 8, r = nb % 8, xcd = bid % 8;
    return xcd * q + (xcd < r ? xcd : r) + bid / 8;
}

// The epilogue of one output point pt (rhs rhs) of parity par: out = a x + b acc
// (twists, in-place CG residual update and norm as selected); returns the point's
// contribution to the norm (EPI_NORM), else 0.
template <int SP, int EPI, bool NT>
__device__ __forceinline__ double hop_epilogue(const HopArgs &a, int par, long pt, int rhs,
                                               cpx<typename SpinorIO<SP>::real> acc[12]) {
    using T = typename SpinorIO<SP>::real;
    double nrm = 0.0;
    const T b = (T)a.b;
    if (a.tm_h != 0.0) twist<T, 12>(acc, 0, (T)a.tm_h);
    if constexpr (EPI & EPI_XPAY) {
        cpx<T> xv[12];
        SpinorIO<SP>::load(a.x[par], pt, xv);
        if (a.tm_x != 0.0) twist<T, 12>(xv, 0, (T)a.tm_x);
        const T aa = (T)a.a;
#pragma unroll
        for (int k = 0; k < 12; ++k)
            acc[k] = {fma(b, acc[k].re, aa * xv[k].re), fma(b, acc[k].im, aa * xv[k].im)};
    } else {
#pragma unroll
        for (int k = 0; k < 12; ++k) acc[k] = b * acc[k];
    }
    if constexpr (EPI & EPI_CGR) {
        // r -= alpha y in place, ||r||^2 (y itself is not stored)
        const double alpha = *(const double *)(a.alpha + (long)rhs * a.alpha_stride);
        if (alpha == 0.0) return nrm;
        cpx<T> rv[12];
        SpinorIO<SP>::load(a.r[par], pt, rv);
        const T al = (T)alpha;
#pragma unroll
        for (int k = 0; k < 12; ++k) rv[k] = {fma(-al, acc[k].re, rv[k].re), fma(-al, acc[k].im, rv[k].im)};
        SpinorIO<SP>::store(a.r[par], pt, rv);
        if constexpr (SP != WL_F64) SpinorIO<SP>::load(a.r[par], pt, rv);
#pragma unroll
        for (int k = 0; k < 12; ++k) nrm += (double)rv[k].re * rv[k].re + (double)rv[k].im * rv[k].im;
        return nrm;
    }
    SpinorIO<SP>::template store<NT && !(EPI & EPI_CACHED_OUT)>(a.out[par], pt, acc);
    if constexpr (EPI & EPI_NORM) {
        if constexpr (SP == WL_F64) {
#pragma unroll
            for (int k = 0; k < 12; ++k) nrm += acc[k].re * acc[k].re + acc[k].im * acc[k].im;
        } else {
            // the norm of what was stored (after rounding to the storage format)
            cpx<T> st[12];
            SpinorIO<SP>::load(a.out[par], pt, st);
#pragma unroll
            for (int k = 0; k < 12; ++k) nrm += (double)st[k].re * st[k].re + (double)st[k].im * st[k].im;
        }
    }
    return nrm;
}

// The work of one thread of the one-thread-per-point kernels: output point at
// position gid of the processing order of parity par.  Returns the point's
// contribution to ||out||^2 (EPI_NORM), else 0.
template <int SP, int GP, int RECON, bool DAG, int EPI, bool NT>
__device__ __forceinline__ double hop_point(const HopArgs &a, int par, long gid) {
    using T = typename SpinorIO<SP>::real;
    double nrm = 0.0;
    if (gid >= a.npts) return nrm;
    int rhs;
    const int i = site_of(a, pos_of_point(a, gid, rhs));
    const long pt = (long)i * a.nrhs + rhs;
    int c[4];
    eo_coords(a.g, i, par, c);
    const int xh = c[0] >> 1;
    cpx<T> acc[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] = {T(0), T(0)};
    hop<SP, GP, RECON, DAG, NT, 0, true>(a, par, i, xh, c, rhs, acc);
    hop<SP, GP, RECON, DAG, NT, 0, false>(a, par, i, xh, c, rhs, acc);
    hop<SP, GP, RECON, DAG, NT, 1, true>(a, par, i, xh, c, rhs, acc);
    hop<SP, GP, RECON, DAG, NT, 1, false>(a, par, i, xh, c, rhs, acc);
    hop<SP, GP, RECON, DAG, NT, 2, true>(a, par, i, xh, c, rhs, acc);
    hop<SP, GP, RECON, DAG, NT, 2, false>(a, par, i, xh, c, rhs, acc);
    hop<SP, GP, RECON, DAG, NT, 3, true>(a, par, i, xh, c, rhs, acc);
    hop<SP, GP, RECON, DAG, NT, 3, false>(a, par, i, xh, c, rhs, acc);
    return hop_epilogue<SP, EPI, NT>(a, par, pt, rhs, acc);
}

// One thread per output point.
template <int SP, int GP, int RECON, bool DAG, int EPI, bool NT>
__global__ void __launch_bounds__(256) hop_kernel(const HopArgs a) {
    if (a.flag && *a.flag == 0) return;
    const int par = a.out_par0 + blockIdx.y;
    const long lb = logical_block(a.swizzle);
    const long gid = lb * blockDim.x + threadIdx.x;  // position in the processing order
    const double nrm = hop_point<SP, GP, RECON, DAG, EPI, NT>(a, par, gid);
    if constexpr (EPI & EPI_NORM) {
        __shared__ double lds[256];
        const long blk = (long)blockIdx.y * gridDim.x + lb;
        block_sum_rhs(nrm, gid, a.nrhs, lds, a.partials + blk, a.part_stride);
    }
}

// Time sweep: a thread owns one point (q, rhs) of a time slice (q the site's
// index within its slice) and walks `sweep` consecutive slices t0 .. t0+sweep-1.
// The input spinors of its own column at t-1, t and t+1 stay in registers, so
// each is read from memory once per sweep and serves both time hops (and the
// x hop inside the site pair) without a cache; the y, z and other x neighbours
// are the loads of neighbouring threads and blocks at the same t.  Blocks tile
// the points of a slice (rhs fastest); consecutive blocks take consecutive tiles
// of the same time range, so with the XCD swizzle each XCD sweeps a contiguous
// range of positions and finds its z neighbours in its own L2.  The arithmetic
// of each output point is that of the one-thread-per-point kernel, bit for bit.
template <int SP, int GP, int RECON, bool DAG, int EPI, bool NT>
__global__ void __launch_bounds__(256) hop_sweep_kernel(const HopArgs a) {
    using T = typename SpinorIO<SP>::real;
    if (a.flag && *a.flag == 0) return;
    const int par = a.out_par0 + blockIdx.y;
    const Geom &g = a.g;
    const long S = g.st;                       // sites per time slice of one parity
    const long spts = S * a.nrhs;              // points per slice
    const long ntile = (spts + blockDim.x - 1) / blockDim.x;
    const long lb = logical_block(a.swizzle);  // gridDim.x = ntile * time ranges
    const long tile = lb % ntile, range = lb / ntile;
    const int t0 = (int)range * a.sweep, t1 = min(g.L[3], t0 + a.sweep);
    const long sp = tile * blockDim.x + threadIdx.x;
    double nrm = 0.0;
    if (sp < spts && t0 < t1) {
        int rhs;
        const long q = pos_of_point(a, sp, rhs);
        const void *in = a.in[1 - par];
        const int lt = g.L[3];
        cpx<T> fm[12], f0[12], fp[12];  // input of this column at t - 1, t, t + 1 (and their factors)
        T sm = load_nb<SP>(in, (q + (long)((t0 - 1 + lt) % lt) * S) * a.nrhs + rhs, fm);
        T s0 = load_nb<SP>(in, (q + (long)t0 * S) * a.nrhs + rhs, f0);
        T sp_ = load_nb<SP>(in, (q + (long)((t0 + 1) % lt) * S) * a.nrhs + rhs, fp);
        for (int t = t0; t < t1; ++t) {
            const int i = (int)(q + (long)t * S);
            int c[4];
            eo_coords(g, i, par, c);
            const int xh = c[0] >> 1;
            cpx<T> acc[12], f[12];
#pragma unroll
            for (int k = 0; k < 12; ++k) acc[k] = {T(0), T(0)};
            int j;
            bool wrap;
            T sf;
            // x: one of the two neighbours is the other site of the pair (index i, f0)
            hop_neighbour<0, true>(g, i, xh, c, j, wrap);
            if (j == i) {
#pragma unroll
                for (int k = 0; k < 12; ++k) f[k] = f0[k];
                sf = s0;
            } else {
                sf = load_nb<SP>(in, (long)j * a.nrhs + rhs, f);
            }
            hop_apply<SP, GP, RECON, DAG, NT, 0, true>(a, par, i, j, wrap, f, sf, acc);
            hop_neighbour<0, false>(g, i, xh, c, j, wrap);
            if (j == i) {
#pragma unroll
                for (int k = 0; k < 12; ++k) f[k] = f0[k];
                sf = s0;
            } else {
                sf = load_nb<SP>(in, (long)j * a.nrhs + rhs, f);
            }
            hop_apply<SP, GP, RECON, DAG, NT, 0, false>(a, par, i, j, wrap, f, sf, acc);
            hop<SP, GP, RECON, DAG, NT, 1, true>(a, par, i, xh, c, rhs, acc);
            hop<SP, GP, RECON, DAG, NT, 1, false>(a, par, i, xh, c, rhs, acc);
            hop<SP, GP, RECON, DAG, NT, 2, true>(a, par, i, xh, c, rhs, acc);
            hop<SP, GP, RECON, DAG, NT, 2, false>(a, par, i, xh, c, rhs, acc);
            // t: the column's own inputs at t + 1 and t - 1
            hop_neighbour<3, true>(g, i, xh, c, j, wrap);
            hop_apply<SP, GP, RECON, DAG, NT, 3, true>(a, par, i, j, wrap, fp, sp_, acc);
            hop_neighbour<3, false>(g, i, xh, c, j, wrap);
            hop_apply<SP, GP, RECON, DAG, NT, 3, false>(a, par, i, j, wrap, fm, sm, acc);
            nrm += hop_epilogue<SP, EPI, NT>(a, par, (long)i * a.nrhs + rhs, rhs, acc);
            if (t + 1 < t1) {
#pragma unroll
                for (int k = 0; k < 12; ++k) {
                    fm[k] = f0[k];
                    f0[k] = fp[k];
                }
                sm = s0;
                s0 = sp_;
                sp_ = load_nb<SP>(in, (q + (long)((t + 2) % lt) * S) * a.nrhs + rhs, fp);
            }
        }
    }
    if constexpr (EPI & EPI_NORM) {
        __shared__ double lds[256];
        const long blk = (long)blockIdx.y * gridDim.x + lb;
        block_sum_rhs(nrm, sp, a.nrhs, lds, a.partials + blk, a.part_stride);
    }
}

// R right-hand sides per thread: thread gid takes site position gid / (nrhs / R)
// and right-hand sides R * (gid % (nrhs / R)) ... + R - 1.
template <int SP, int GP, int RECON, bool DAG, int EPI, bool NT, int R>
__global__ void __launch_bounds__(256) hop_kernel_mr(const HopArgs a) {
    using T = typename SpinorIO<SP>::real;
    if (a.flag && *a.flag == 0) return;
    const int par = a.out_par0 + blockIdx.y;
    const long lb = logical_block(a.swizzle);
    const long gid = lb * blockDim.x + threadIdx.x;
    const int G = a.nrhs / R;
    const bool active = gid < a.npts / R;
    double nrm[R];
#pragma unroll
    for (int r = 0; r < R; ++r) nrm[r] = 0.0;
    const int ps = (int)gid / G;
    const int rhs0 = ((int)gid - ps * G) * R;
    if (active) {
        const int i = site_of(a, ps);
        int c[4];
        eo_coords(a.g, i, par, c);
        const int xh = c[0] >> 1;
        cpx<T> acc[R][12];
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int k = 0; k < 12; ++k) acc[r][k] = {T(0), T(0)};
        hop_r<SP, GP, RECON, DAG, NT, 0, true, R>(a, par, i, xh, c, rhs0, acc);
        hop_r<SP, GP, RECON, DAG, NT, 0, false, R>(a, par, i, xh, c, rhs0, acc);
        hop_r<SP, GP, RECON, DAG, NT, 1, true, R>(a, par, i, xh, c, rhs0, acc);
        hop_r<SP, GP, RECON, DAG, NT, 1, false, R>(a, par, i, xh, c, rhs0, acc);
        hop_r<SP, GP, RECON, DAG, NT, 2, true, R>(a, par, i, xh, c, rhs0, acc);
        hop_r<SP, GP, RECON, DAG, NT, 2, false, R>(a, par, i, xh, c, rhs0, acc);
        hop_r<SP, GP, RECON, DAG, NT, 3, true, R>(a, par, i, xh, c, rhs0, acc);
        hop_r<SP, GP, RECON, DAG, NT, 3, false, R>(a, par, i, xh, c, rhs0, acc);
        const T b = (T)a.b;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const long pt = (long)i * a.nrhs + rhs0 + r;
            if (a.tm_h != 0.0) twist<T, 12>(acc[r], 0, (T)a.tm_h);
            if constexpr (EPI & EPI_XPAY) {
                cpx<T> xv[12];
                SpinorIO<SP>::load(a.x[par], pt, xv);
                if (a.tm_x != 0.0) twist<T, 12>(xv, 0, (T)a.tm_x);
                const T aa = (T)a.a;
#pragma unroll
                for (int k = 0; k < 12; ++k)
                    acc[r][k] = {fma(b, acc[r][k].re, aa * xv[k].re), fma(b, acc[r][k].im, aa * xv[k].im)};
            } else {
#pragma unroll
                for (int k = 0; k < 12; ++k) acc[r][k] = b * acc[r][k];
            }
            SpinorIO<SP>::template store<NT>(a.out[par], pt, acc[r]);
            if constexpr (EPI & EPI_NORM) {
                if constexpr (SP == WL_F64) {
#pragma unroll
                    for (int k = 0; k < 12; ++k) nrm[r] += acc[r][k].re * acc[r][k].re + acc[r][k].im * acc[r][k].im;
                } else {
                    cpx<T> st[12];
                    SpinorIO<SP>::load(a.out[par], pt, st);
#pragma unroll
                    for (int k = 0; k < 12; ++k) nrm[r] += (double)st[k].re * st[k].re + (double)st[k].im * st[k].im;
                }
            }
        }
    }
    if constexpr (EPI & EPI_NORM) {
        // per-rhs block sums in a fixed order: entry (thread t, r) belongs to
        // rhs R * ((gid of t) % G) + r
        __shared__ double lds[256 * R];
#pragma unroll
        for (int r = 0; r < R; ++r) lds[threadIdx.x * R + r] = nrm[r];
        __syncthreads();
        const long g0 = lb * blockDim.x;
        if ((int)threadIdx.x < a.nrhs) {
            const int want = threadIdx.x, r = want % R, grp = want / R;
            double s = 0.0;
            for (int t = 0; t < (int)blockDim.x; ++t)
                if ((int)((g0 + t) % G) == grp) s += lds[t * R + r];
            const long blk = (long)blockIdx.y * gridDim.x + lb;
            a.partials[(long)want * a.part_stride + blk] = s;
        }
    }
}

// Two threads per output point: lanes 0-31 of a wavefront take the forward
// hops of 32 consecutive points, lanes 32-63 the backward hops of the same
// points; the partial sums are exchanged across the halves and each half
// finishes and stores two of the four spin components.  The work of one
// thread for logical block lb of parity par; *gid_out = the point's position
// in the processing order.  Returns the thread's share of ||out||^2
// (EPI_NORM), else 0.  Every lane of the wavefront must call it.
template <int SP, int GP, int RECON, bool DAG, int EPI, bool NT>
__device__ __forceinline__ double hop_split_point(const HopArgs &a, int par, long lb, long *gid_out) {
    using T = typename SpinorIO<SP>::real;
    const int lane = threadIdx.x & 63;
    const bool fwd = lane < 32;
    const int hf = fwd ? 0 : 1;  // spin half this lane stores
    const long gid = ((lb * blockDim.x + threadIdx.x) >> 6) * 32 + (lane & 31);
    long pt = 0;
    const bool active = gid < a.npts;
    cpx<T> acc[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] = {T(0), T(0)};
    if (active) {
        int rhs;
        const int i = site_of(a, pos_of_point(a, gid, rhs));
        pt = (long)i * a.nrhs + rhs;
        int c[4];
        eo_coords(a.g, i, par, c);
        const int xh = c[0] >> 1;
        hop_rt<SP, GP, RECON, DAG, NT, 0>(a, par, i, xh, c, rhs, fwd, acc);
        hop_rt<SP, GP, RECON, DAG, NT, 1>(a, par, i, xh, c, rhs, fwd, acc);
        hop_rt<SP, GP, RECON, DAG, NT, 2>(a, par, i, xh, c, rhs, fwd, acc);
        hop_rt<SP, GP, RECON, DAG, NT, 3>(a, par, i, xh, c, rhs, fwd, acc);
    }
    // every lane takes part in the exchange
    cpx<T> res[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const cpx<T> send = fwd ? acc[6 + k] : acc[k];
        const cpx<T> own = fwd ? acc[k] : acc[6 + k];
        const cpx<T> recv = {__shfl_xor(send.re, 32, 64), __shfl_xor(send.im, 32, 64)};
        res[k] = own + recv;
    }
    double nrm = 0.0;
    if (active) {
        const T b = (T)a.b;
        if (a.tm_h != 0.0) twist<T, 6>(res, 6 * hf, (T)a.tm_h);
        if constexpr (EPI & EPI_XPAY) {
            cpx<T> xv[6];
            SpinorIO<SP>::load_half(a.x[par], pt, hf, xv);
            if (a.tm_x != 0.0) twist<T, 6>(xv, 6 * hf, (T)a.tm_x);
            const T aa = (T)a.a;
#pragma unroll
            for (int k = 0; k < 6; ++k)
                res[k] = {fma(b, res[k].re, aa * xv[k].re), fma(b, res[k].im, aa * xv[k].im)};
        } else {
#pragma unroll
            for (int k = 0; k < 6; ++k) res[k] = b * res[k];
        }
    }
    // what is stored where: y = res in out, or (EPI_CGR) r - alpha y in r
    void *dst = a.out[par];
    bool doit = active;
    // the residual is read again at once, and so are cached outputs
    constexpr bool NTS = NT && !(EPI & EPI_CGR) && !(EPI & EPI_CACHED_OUT);
    if constexpr (EPI & EPI_CGR) {
        dst = a.r[par];
        if (active) {
            const double alpha = *(const double *)(a.alpha + (long)((int)gid % a.nrhs) * a.alpha_stride);
            doit = alpha != 0.0;
            if (doit) {
                cpx<T> rv[6];
                SpinorIO<SP>::load_half(a.r[par], pt, hf, rv);
                const T al = (T)alpha;
#pragma unroll
                for (int k = 0; k < 6; ++k) res[k] = {fma(-al, res[k].re, rv[k].re), fma(-al, res[k].im, rv[k].im)};
            }
        }
    }
    if constexpr (SP == WL_F64 || SP == WL_F32) {
        if (doit) {
            SpinorIO<SP>::template store_half<NTS>(dst, pt, hf, res);
            if constexpr (EPI & EPI_NORM) {
                if constexpr (SP != WL_F64) SpinorIO<SP>::load_half(dst, pt, hf, res);
#pragma unroll
                for (int k = 0; k < 6; ++k) nrm += (double)res[k].re * res[k].re + (double)res[k].im * res[k].im;
            }
        }
    } else {
        // 16-bit storage: one norm per point, the largest component of both halves
        float m = 0.f;
        if (doit)
#pragma unroll
            for (int k = 0; k < 6; ++k) m = fmaxf(m, fmaxf(fabsf(res[k].re), fabsf(res[k].im)));
        m = fmaxf(m, __shfl_xor(m, 32, 64));
        if (doit) {
            SpinorIO<SP>::template store_half_shared<NTS>(dst, pt, hf, res, m);
            if constexpr (EPI & EPI_NORM) {
#pragma unroll
                for (int k = 0; k < 6; ++k) nrm += (double)res[k].re * res[k].re + (double)res[k].im * res[k].im;
            }
        }
    }
    *gid_out = gid;
    return nrm;
}

template <int SP, int GP, int RECON, bool DAG, int EPI, bool NT>
__global__ void __launch_bounds__(256) hop_kernel_split(const HopArgs a) {
    if (a.flag && *a.flag == 0) return;
    const int par = a.out_par0 + blockIdx.y;
    const long lb = logical_block(a.swizzle);
    long gid;
    const double nrm = hop_split_point<SP, GP, RECON, DAG, EPI, NT>(a, par, lb, &gid);
    if constexpr (EPI & EPI_NORM) {
        __shared__ double lds[256];
        __shared__ int lrhs[256];
        const long blk = (long)blockIdx.y * gridDim.x + lb;
        block_sum_by_rhs(nrm, (int)gid % a.nrhs, a.nrhs, lds, lrhs, a.partials + blk, a.part_stride);
    }
}

// Persistent launch over the tiles of all systems: the tile list is cut into
// eight contiguous ranges, one per XCD (the hardware places workgroup b on XCD
// b mod 8), and the workgroups of an XCD take its tiles round-robin.  Every tile
// costs the same, so a static schedule balances as well as a shared counter
// would, without serialising every claim on one atomic address.  The tile index
// is derived from blockIdx only, so all control flow around the barriers of the
// norm epilogue is uniform.
template <int SP, int GP, int RECON, bool DAG, int EPI, bool NT, int TPS>
__global__ void __launch_bounds__(256) hop_batch_kernel(const BatchArgs B) {
    __shared__ double lds[256];
    __shared__ int lrhs[TPS == 2 ? 256 : 1];
    const int xcd = blockIdx.x % 8, j = blockIdx.x / 8, nper = gridDim.x / 8;  // gridDim.x: a multiple of 8
    const int r0 = (int)(B.ntiles * xcd / 8), r1 = (int)(B.ntiles * (xcd + 1) / 8);
    for (int tile = r0 + j; tile < r1; tile += nper) {
        int sy = 0;
        while (sy + 1 < B.nsys && tile >= B.start[sy + 1]) ++sy;
        const HopArgs &a = B.sys[sy];
        // tiles of a system that has stopped iterating are skipped
        const int live = a.flag ? __builtin_amdgcn_readfirstlane(*a.flag) : 1;
        if (live != 0) {
            const long local = tile - B.start[sy];
            const int py = (int)(local / B.per_par[sy]);
            const long lb = local - (long)py * B.per_par[sy];
            if constexpr (TPS == 2) {
                long gid;
                const double nrm = hop_split_point<SP, GP, RECON, DAG, EPI, NT>(a, a.out_par0 + py, lb, &gid);
                if constexpr (EPI & EPI_NORM)
                    block_sum_by_rhs(nrm, (int)gid % a.nrhs, a.nrhs, lds, lrhs, a.partials + local, a.part_stride);
            } else {
                const long gid = lb * blockDim.x + threadIdx.x;
                const double nrm = hop_point<SP, GP, RECON, DAG, EPI, NT>(a, a.out_par0 + py, gid);
                if constexpr (EPI & EPI_NORM) block_sum_rhs(nrm, gid, a.nrhs, lds, a.partials + local, a.part_stride);
            }
        }
    }
}


// Launch of the R-right-hand-sides-per-thread kernel for every storage format,
// dagger, epilogue and non-temporal choice; instantiated once per R in its own
// translation unit (wl_dslash_r2/3/4.hip) to keep compile times short.
template <int SP, int GP, int RECON, bool DAG, bool NT, int R>
static hipError_t launch_r_epi(int epi, const HopArgs &a, dim3 grid, dim3 blk, hipStream_t s) {
    switch (epi) {
    case 0: hipLaunchKernelGGL((hop_kernel_mr<SP, GP, RECON, DAG, 0, NT, R>), grid, blk, a.shm, s, a); break;
    case EPI_XPAY: hipLaunchKernelGGL((hop_kernel_mr<SP, GP, RECON, DAG, EPI_XPAY, NT, R>), grid, blk, a.shm, s, a); break;
    case EPI_NORM: hipLaunchKernelGGL((hop_kernel_mr<SP, GP, RECON, DAG, EPI_NORM, NT, R>), grid, blk, a.shm, s, a); break;
    case EPI_XPAY | EPI_NORM:
        hipLaunchKernelGGL((hop_kernel_mr<SP, GP, RECON, DAG, EPI_XPAY | EPI_NORM, NT, R>), grid, blk, a.shm, s, a);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int SP, int GP, int RECON, int R>
static hipError_t launch_r_dag(bool dag, bool nt, int epi, const HopArgs &a, dim3 grid, dim3 blk, hipStream_t s) {
    if (nt)
        return dag ? launch_r_epi<SP, GP, RECON, true, true, R>(epi, a, grid, blk, s)
                   : launch_r_epi<SP, GP, RECON, false, true, R>(epi, a, grid, blk, s);
    return dag ? launch_r_epi<SP, GP, RECON, true, false, R>(epi, a, grid, blk, s)
               : launch_r_epi<SP, GP, RECON, false, false, R>(epi, a, grid, blk, s);
}

template <int R>
static hipError_t launch_hop_r_impl(int prec, int recon, bool dag, bool nt, int epi, const HopArgs &a, dim3 grid,
                                    dim3 blk, hipStream_t s) {
    if (prec == WL_F64)
        return recon == 12 ? launch_r_dag<WL_F64, WL_F64, 12, R>(dag, nt, epi, a, grid, blk, s)
                           : launch_r_dag<WL_F64, WL_F64, 18, R>(dag, nt, epi, a, grid, blk, s);
    if (prec == WL_F32)
        return recon == 12 ? launch_r_dag<WL_F32, WL_F32, 12, R>(dag, nt, epi, a, grid, blk, s)
                           : launch_r_dag<WL_F32, WL_F32, 18, R>(dag, nt, epi, a, grid, blk, s);
    if (prec == WL_F16N && recon == 12) return launch_r_dag<WL_F16N, WL_F16N, 12, R>(dag, nt, epi, a, grid, blk, s);
    if (prec == WL_BF16N && recon == 12) return launch_r_dag<WL_BF16N, WL_BF16N, 12, R>(dag, nt, epi, a, grid, blk, s);
    if (prec == WL_I16N && recon == 12) return launch_r_dag<WL_I16N, WL_I16N, 12, R>(dag, nt, epi, a, grid, blk, s);
    return hipErrorInvalidValue;
}

// defined in wl_dslash_r2.hip, wl_dslash_r3.hip, wl_dslash_r4.hip
hipError_t launch_hop_r2(int prec, int recon, bool dag, bool nt, int epi, const HopArgs &a, dim3 grid, dim3 blk,
                         hipStream_t s);
hipError_t launch_hop_r3(int prec, int recon, bool dag, bool nt, int epi, const HopArgs &a, dim3 grid, dim3 blk,
                         hipStream_t s);
hipError_t launch_hop_r4(int prec, int recon, bool dag, bool nt, int epi, const HopArgs &a, dim3 grid, dim3 blk,
                         hipStream_t s);

}  // namespace wl
