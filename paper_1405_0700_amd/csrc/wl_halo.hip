// Bulk / boundary split of the hopping term with t-face packing (see wl_halo.h).
#include "wl_halo.h"
#include "wl_dslash_kernels.h"

namespace wl {

// One thread per face site f: the forward face is the t = 0 slice of the source
// parity projected for the forward t hop; the backward face is the t = Lt - 1
// slice projected for the backward hop and multiplied by U_t^+ of its site.
template <int SP, int GP, int RECON, bool DAG>
__global__ void __launch_bounds__(256) k_face_pack(const HopArgs a, int par,
                                                   cpx<typename SpinorIO<SP>::real> *fwd,
                                                   cpx<typename SpinorIO<SP>::real> *bwd) {
    using T = typename SpinorIO<SP>::real;
    const long fs = a.g.st;
    const long f = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= fs) return;
    {
        constexpr int S = DAG ? 1 : -1;  // forward hop
        cpx<T> v[12], h[6];
        SpinorIO<SP>::load(a.in[1 - par], f, v);
        project<T, 3, S>(v, h);
#pragma unroll
        for (int k = 0; k < 6; ++k) fwd[k * fs + f] = h[k];
    }
    {
        constexpr int S = DAG ? -1 : 1;  // backward hop
        const long j = (long)(a.g.L[3] - 1) * fs + f;
        cpx<T> v[12], h[6], u[9], w[6];
        SpinorIO<SP>::load(a.in[1 - par], j, v);
        const char *slab = (const char *)a.gauge + (size_t)((1 - par) * 4 + 3) * a.slab_bytes;
        LinkIO<GP, RECON>::template load<false>(slab, (int)j, u);
        project<T, 3, S>(v, h);
        su3_mul2<T, false>(u, h, w);
#pragma unroll
        for (int k = 0; k < 6; ++k) bwd[k * fs + f] = w[k];
    }
}

// One thread per output site (in the launch's processing order): the spatial
// hops and the t hops that stay in the local volume.  Interior slices are finished (scaled and stored); the two
// boundary slices store their partial sums, cut where the fused order reaches
// the first hop through a face (before t+ on the last slice, before t- on the
// first).
template <int SP, int GP, int RECON, bool DAG, bool NT>
__global__ void __launch_bounds__(256) k_hop_bulk(const HopArgs a, int par) {
    using T = typename SpinorIO<SP>::real;
    const long ps = logical_block(a.swizzle) * blockDim.x + threadIdx.x;
    if (ps >= a.npts) return;
    const long i = site_of(a, (int)ps);
    int c[4];
    eo_coords(a.g, (int)i, par, c);
    const int xh = c[0] >> 1, lt = a.g.L[3];
    const bool first = c[3] == 0, last = c[3] == lt - 1;
    cpx<T> acc[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] = {T(0), T(0)};
    hop<SP, GP, RECON, DAG, NT, 0, true>(a, par, (int)i, xh, c, 0, acc);
    hop<SP, GP, RECON, DAG, NT, 0, false>(a, par, (int)i, xh, c, 0, acc);
    hop<SP, GP, RECON, DAG, NT, 1, true>(a, par, (int)i, xh, c, 0, acc);
    hop<SP, GP, RECON, DAG, NT, 1, false>(a, par, (int)i, xh, c, 0, acc);
    hop<SP, GP, RECON, DAG, NT, 2, true>(a, par, (int)i, xh, c, 0, acc);
    hop<SP, GP, RECON, DAG, NT, 2, false>(a, par, (int)i, xh, c, 0, acc);
    if (!last) hop<SP, GP, RECON, DAG, NT, 3, true>(a, par, (int)i, xh, c, 0, acc);
    if (first || last) {
        SpinorIO<SP>::template store<NT>(a.out[par], i, acc);
        return;
    }
    hop<SP, GP, RECON, DAG, NT, 3, false>(a, par, (int)i, xh, c, 0, acc);
    const T b = (T)a.b;
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] = b * acc[k];
    SpinorIO<SP>::template store<NT>(a.out[par], i, acc);
}

// One thread per boundary site (first the t = 0 slice, then t = Lt - 1): the
// partial sum from the output, the hops through the faces (with the boundary
// phase of t) and, on the last slice, the local t- hop after the t+ one.
template <int SP, int GP, int RECON, bool DAG>
__global__ void __launch_bounds__(256) k_hop_boundary(const HopArgs a, int par,
                                                      const cpx<typename SpinorIO<SP>::real> *rfwd,
                                                      const cpx<typename SpinorIO<SP>::real> *rbwd) {
    using T = typename SpinorIO<SP>::real;
    const long fs = a.g.st;
    const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= 2 * fs) return;
    const int lt = a.g.L[3];
    const long f = q < fs ? q : q - fs;
    const long i = q < fs ? f : (long)(lt - 1) * fs + f;
    int c[4];
    eo_coords(a.g, (int)i, par, c);
    const int xh = c[0] >> 1;
    const bool phased = (a.g.phase_mask >> 3) & 1;
    cpx<T> acc[12];
    SpinorIO<SP>::load(a.out[par], i, acc);
    if (c[3] == lt - 1) {
        constexpr int S = DAG ? 1 : -1;  // forward hop through the face
        cpx<T> h[6], u[9], v[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) h[k] = rfwd[k * fs + f];
        const char *slab = (const char *)a.gauge + (size_t)(par * 4 + 3) * a.slab_bytes;
        LinkIO<GP, RECON>::template load<false>(slab, (int)i, u);
        su3_mul2<T, true>(u, h, v);
        if (phased) {
            const cpx<T> z = {(T)a.g.zr[3], (T)a.g.zi[3]};
#pragma unroll
            for (int k = 0; k < 6; ++k) v[k] = cmul(z, v[k]);
        }
        accumulate<T, 3, S>(acc, v, T(1));
        if (c[3] != 0) hop<SP, GP, RECON, DAG, false, 3, false>(a, par, (int)i, xh, c, 0, acc);
    }
    if (c[3] == 0) {
        constexpr int S = DAG ? -1 : 1;  // backward hop through the face
        cpx<T> v[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) v[k] = rbwd[k * fs + f];
        if (phased) {
            const cpx<T> z = {(T)a.g.zr[3], -(T)a.g.zi[3]};
#pragma unroll
            for (int k = 0; k < 6; ++k) v[k] = cmul(z, v[k]);
        }
        accumulate<T, 3, S>(acc, v, T(1));
    }
    const T b = (T)a.b;
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] = b * acc[k];
    SpinorIO<SP>::template store<false>(a.out[par], i, acc);
}

// ------------------------------------------------------------------ launchers
template <int SP, int GP, int RECON>
static hipError_t pack_t(bool dag, const HopArgs &a, int par, void *f, void *b, hipStream_t s) {
    using C = cpx<typename SpinorIO<SP>::real>;
    const dim3 grid((unsigned)((a.g.st + 255) / 256)), blk(256);
    if (dag) hipLaunchKernelGGL((k_face_pack<SP, GP, RECON, true>), grid, blk, 0, s, a, par, (C *)f, (C *)b);
    else hipLaunchKernelGGL((k_face_pack<SP, GP, RECON, false>), grid, blk, 0, s, a, par, (C *)f, (C *)b);
    return hipGetLastError();
}
template <int SP, int GP, int RECON>
static hipError_t bulk_t(bool dag, bool nt, const HopArgs &a, int par, hipStream_t s) {
    const dim3 grid((unsigned)((a.npts + 255) / 256)), blk(256);
    if (dag && nt) hipLaunchKernelGGL((k_hop_bulk<SP, GP, RECON, true, true>), grid, blk, 0, s, a, par);
    else if (dag) hipLaunchKernelGGL((k_hop_bulk<SP, GP, RECON, true, false>), grid, blk, 0, s, a, par);
    else if (nt) hipLaunchKernelGGL((k_hop_bulk<SP, GP, RECON, false, true>), grid, blk, 0, s, a, par);
    else hipLaunchKernelGGL((k_hop_bulk<SP, GP, RECON, false, false>), grid, blk, 0, s, a, par);
    return hipGetLastError();
}
template <int SP, int GP, int RECON>
static hipError_t bound_t(bool dag, const HopArgs &a, int par, const void *f, const void *b, hipStream_t s) {
    using C = cpx<typename SpinorIO<SP>::real>;
    const dim3 grid((unsigned)((2 * a.g.st + 255) / 256)), blk(256);
    if (dag)
        hipLaunchKernelGGL((k_hop_boundary<SP, GP, RECON, true>), grid, blk, 0, s, a, par, (const C *)f, (const C *)b);
    else
        hipLaunchKernelGGL((k_hop_boundary<SP, GP, RECON, false>), grid, blk, 0, s, a, par, (const C *)f,
                           (const C *)b);
    return hipGetLastError();
}

#define WL_HALO_DISPATCH(FN, ...)                                                                        \
    if (prec == WL_F64) return recon == 12 ? FN<WL_F64, WL_F64, 12>(__VA_ARGS__) : FN<WL_F64, WL_F64, 18>(__VA_ARGS__); \
    if (prec == WL_F32) return recon == 12 ? FN<WL_F32, WL_F32, 12>(__VA_ARGS__) : FN<WL_F32, WL_F32, 18>(__VA_ARGS__); \
    return hipErrorInvalidValue;

hipError_t launch_face_pack(int prec, int recon, bool dag, const HopArgs &a, int par, void *send_fwd, void *send_bwd,
                            hipStream_t s) {
    WL_HALO_DISPATCH(pack_t, dag, a, par, send_fwd, send_bwd, s)
}
hipError_t launch_hop_bulk(int prec, int recon, bool dag, bool nt, const HopArgs &a, int par, hipStream_t s) {
    if (a.npts > (1L << 30)) return hipErrorInvalidValue;  // 32-bit point indices
    WL_HALO_DISPATCH(bulk_t, dag, nt, a, par, s)
}
hipError_t launch_hop_boundary(int prec, int recon, bool dag, const HopArgs &a, int par, const void *recv_fwd,
                               const void *recv_bwd, hipStream_t s) {
    WL_HALO_DISPATCH(bound_t, dag, a, par, recv_fwd, recv_bwd, s)
}

}  // namespace wl
