// Wilson hopping term on gfx950: the half-spinor form of Eq. (2).
//
// One thread computes one output point (site, rhs).  For each of the 8 hops it
// loads the neighbouring spinor, projects it onto the two independent spin
// components (the projector (1 -/+ gamma_mu) has rank 2, and in the chiral
// basis its lower two rows are -/+ A_mu^+ times its upper two, Sec. 2 after
// Eq. (2)), multiplies the two colour vectors by U_mu(x) or U_mu(x - mu)^+,
// applies the boundary phase if the hop wraps, and accumulates the upper
// components and the rebuilt lower ones.  The projected half spinors live in
// registers only; nothing but the input spinor, the links and the output point
// touches HBM.
//
// The kernel is bandwidth-bound (about 1 flop per byte in FP64), so it is laid
// out for coalescing: every field is structure-of-arrays with the point index
// fastest, consecutive threads handle consecutive points, and consecutive
// blocks are optionally remapped so that each XCD (which has its own L2) works
// on one contiguous range of sites and the neighbour re-reads hit its L2.
#include "wl_dslash.h"

namespace wl {

// -i a
template <typename T> __device__ __forceinline__ cpx<T> mi(cpx<T> a) { return {a.im, -a.re}; }

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

// acc_up += v ; acc_lo += S * A_mu^+ v.
// A_x^+ v = (i v1, i v0), A_y^+ v = (v1, -v0), A_z^+ v = (i v0, -i v1), A_t^+ v = -v.
template <typename T, int MU, int S>
__device__ __forceinline__ void accumulate(cpx<T> acc[12], const cpx<T> v[6]) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const cpx<T> v0 = v[c], v1 = v[3 + c];
        acc[c] = acc[c] + v0;
        acc[3 + c] = acc[3 + c] + v1;
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
        if constexpr (S > 0) {
            acc[6 + c] = acc[6 + c] + w0;
            acc[9 + c] = acc[9 + c] + w1;
        } else {
            acc[6 + c] = acc[6 + c] - w0;
            acc[9 + c] = acc[9 + c] - w1;
        }
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

template <int SP, int GP, int RECON, bool DAG, int MU, bool FWD>
__device__ __forceinline__ void hop(const HopArgs &a, int par, int i, int xh, const int c[4], int rhs,
                                    cpx<typename SpinorIO<SP>::real> acc[12]) {
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
    // Forward hop (H): (1 - gamma) -> S = -1; backward: (1 + gamma) -> S = +1; H^+ swaps them.
    constexpr int S = (FWD != DAG) ? -1 : 1;
    cpx<T> f[12], h[6], u[9], v[6];
    SpinorIO<SP>::load(a.in[1 - par], a.npts, (long)j * a.nrhs + rhs, f);
    const int lpar = FWD ? par : 1 - par;
    const char *slab = (const char *)a.gauge + (size_t)(lpar * 4 + MU) * a.slab_bytes;
    LinkIO<GP, RECON>::load(slab, g.vh, FWD ? i : j, u);
    project<T, MU, S>(f, h);
    su3_mul2<T, FWD>(u, h, v);
    if (wrap && ((g.phase_mask >> MU) & 1)) {
        const cpx<T> z = {(T)g.zr[MU], FWD ? (T)g.zi[MU] : -(T)g.zi[MU]};
#pragma unroll
        for (int k = 0; k < 6; ++k) v[k] = cmul(z, v[k]);
    }
    accumulate<T, MU, S>(acc, v);
}

__device__ __forceinline__ long logical_block(int swizzle) {
    const long nb = gridDim.x, bid = blockIdx.x;
    if (!swizzle || nb < 16) return bid;
    // hardware dispatches block b to XCD b % 8: give XCD x one contiguous range
    const long q = nb / 8, r = nb % 8, xcd = bid % 8;
    return xcd * q + (xcd < r ? xcd : r) + bid / 8;
}

template <int SP, int GP, int RECON, bool DAG, int EPI>
__global__ void __launch_bounds__(256) hop_kernel(const HopArgs a) {
    using T = typename SpinorIO<SP>::real;
    if (a.flag && *a.flag) return;
    const int par = a.out_par0 + blockIdx.y;
    const long lb = logical_block(a.swizzle);
    const long gid = lb * blockDim.x + threadIdx.x;
    const bool active = gid < a.npts;
    double nrm = 0.0;
    int rhs = 0;
    if (active) {
        const int i = (int)(gid / a.nrhs);
        rhs = (int)(gid - (long)i * a.nrhs);
        int c[4];
        eo_coords(a.g, i, par, c);
        const int xh = c[0] >> 1;
        cpx<T> acc[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) acc[k] = {T(0), T(0)};
        hop<SP, GP, RECON, DAG, 0, true>(a, par, i, xh, c, rhs, acc);
        hop<SP, GP, RECON, DAG, 0, false>(a, par, i, xh, c, rhs, acc);
        hop<SP, GP, RECON, DAG, 1, true>(a, par, i, xh, c, rhs, acc);
        hop<SP, GP, RECON, DAG, 1, false>(a, par, i, xh, c, rhs, acc);
        hop<SP, GP, RECON, DAG, 2, true>(a, par, i, xh, c, rhs, acc);
        hop<SP, GP, RECON, DAG, 2, false>(a, par, i, xh, c, rhs, acc);
        hop<SP, GP, RECON, DAG, 3, true>(a, par, i, xh, c, rhs, acc);
        hop<SP, GP, RECON, DAG, 3, false>(a, par, i, xh, c, rhs, acc);
        const T b = (T)a.b;
        if constexpr (EPI & EPI_XPAY) {
            cpx<T> xv[12];
            SpinorIO<SP>::load(a.x[par], a.npts, gid, xv);
            const T aa = (T)a.a;
#pragma unroll
            for (int k = 0; k < 12; ++k)
                acc[k] = {fma(b, acc[k].re, aa * xv[k].re), fma(b, acc[k].im, aa * xv[k].im)};
        } else {
#pragma unroll
            for (int k = 0; k < 12; ++k) acc[k] = b * acc[k];
        }
        SpinorIO<SP>::store(a.out[par], a.npts, gid, acc);
        if constexpr (EPI & EPI_NORM) {
            if constexpr (SP == WL_F64) {
#pragma unroll
                for (int k = 0; k < 12; ++k) nrm += acc[k].re * acc[k].re + acc[k].im * acc[k].im;
            } else {
                // the norm of what was stored (after rounding to the storage format)
                cpx<T> st[12];
                SpinorIO<SP>::load(a.out[par], a.npts, gid, st);
#pragma unroll
                for (int k = 0; k < 12; ++k)
                    nrm += (double)st[k].re * st[k].re + (double)st[k].im * st[k].im;
            }
        }
    }
    if constexpr (EPI & EPI_NORM) {
        __shared__ double lds[256];
        const long blk = (long)blockIdx.y * gridDim.x + lb;
        block_sum_rhs(nrm, gid, a.nrhs, lds, a.partials + blk, a.part_stride);
    }
}

template <int SP, int GP, int RECON, bool DAG>
static hipError_t launch_epi(int epi, HopArgs &a, dim3 grid, dim3 block, hipStream_t s) {
    switch (epi) {
    case 0: hipLaunchKernelGGL((hop_kernel<SP, GP, RECON, DAG, 0>), grid, block, 0, s, a); break;
    case EPI_XPAY: hipLaunchKernelGGL((hop_kernel<SP, GP, RECON, DAG, EPI_XPAY>), grid, block, 0, s, a); break;
    case EPI_NORM: hipLaunchKernelGGL((hop_kernel<SP, GP, RECON, DAG, EPI_NORM>), grid, block, 0, s, a); break;
    case EPI_XPAY | EPI_NORM:
        hipLaunchKernelGGL((hop_kernel<SP, GP, RECON, DAG, EPI_XPAY | EPI_NORM>), grid, block, 0, s, a);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int SP, int GP, int RECON>
static hipError_t launch_dag(bool dag, int epi, HopArgs &a, dim3 grid, dim3 block, hipStream_t s) {
    return dag ? launch_epi<SP, GP, RECON, true>(epi, a, grid, block, s)
               : launch_epi<SP, GP, RECON, false>(epi, a, grid, block, s);
}

hipError_t launch_hop(int prec, int recon, bool dagger, int epi, HopArgs &a, int nparity,
                      const LaunchCfg &cfg, hipStream_t stream) {
    const int block = cfg.block;
    if (block <= 0 || block > 256 || block % 64) return hipErrorInvalidValue;
    a.swizzle = cfg.swizzle;
    dim3 grid((unsigned)hop_blocks(a.npts, block), (unsigned)nparity);
    dim3 blk(block);
    if (prec == WL_F64)
        return recon == 12 ? launch_dag<WL_F64, WL_F64, 12>(dagger, epi, a, grid, blk, stream)
                           : launch_dag<WL_F64, WL_F64, 18>(dagger, epi, a, grid, blk, stream);
    if (prec == WL_F32)
        return recon == 12 ? launch_dag<WL_F32, WL_F32, 12>(dagger, epi, a, grid, blk, stream)
                           : launch_dag<WL_F32, WL_F32, 18>(dagger, epi, a, grid, blk, stream);
    if (prec == WL_F16N && recon == 12) return launch_dag<WL_F16N, WL_F16N, 12>(dagger, epi, a, grid, blk, stream);
    if (prec == WL_BF16N && recon == 12) return launch_dag<WL_BF16N, WL_BF16N, 12>(dagger, epi, a, grid, blk, stream);
    return hipErrorInvalidValue;
}

}  // namespace wl
