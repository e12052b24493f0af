// Parallel-transport convolution (PTC) preconditioner on gfx950.
//
// A layer maps C_in spinor fields to C_out spinor fields through nine paths
// (the identity and the eight one-hop transports U_mu(x) psi(x+mu),
// U_mu(x-mu)^+ psi(x-mu), with the Wilson operator's boundary phases), each
// followed by a complex 4x4 spin matrix per (output, input) channel pair.  The
// spin matrices commute with the transports, so a thread first mixes the input
// channels at the neighbour site and then transports the mixed spinor once per
// path.  Fields are FP32, channel-major (each channel a FULL field, so a
// wave's threads, one per site, read consecutive points of a channel); weights
// are read from BF16 (or FP32) and staged as FP32 in LDS; accumulation is FP32.
#include "wl_ptc.h"

namespace wl {

__device__ __forceinline__ int ptc_reverse(int q) { return q == 0 ? 0 : (((q - 1) & 1) ? q - 1 : q + 1); }

// neighbour of even/odd site i (parity par, coordinates c) along path q:
// returns its index j and parity, whether the hop wraps, and the link
// (parity, index) the transport uses
struct PathHop {
    int j, npar, lpar, lsite, mu;
    bool fwd, wrap;
};
__device__ __forceinline__ PathHop ptc_hop(const Geom &g, int i, int par, const int c[4], int q) {
    PathHop h;
    if (q == 0) {
        h.j = i;
        h.npar = par;
        h.mu = -1;
        h.fwd = true;
        h.wrap = false;
        h.lpar = 0;
        h.lsite = 0;
        return h;
    }
    const int mu = (q - 1) >> 1;
    const bool fwd = ((q - 1) & 1) == 0;
    int j;
    bool wrap;
    if (mu == 0) {
        int x = c[0] + (fwd ? 1 : -1);
        wrap = fwd ? (x == g.L[0]) : (x < 0);
        if (wrap) x = fwd ? 0 : g.L[0] - 1;
        j = (i - (c[0] >> 1)) + (x >> 1);
    } else {
        const int stride = mu == 1 ? g.sy : (mu == 2 ? g.sz : g.st);
        wrap = fwd ? (c[mu] == g.L[mu] - 1) : (c[mu] == 0);
        j = fwd ? i + stride : i - stride;
        if (wrap) j += fwd ? -g.L[mu] * stride : g.L[mu] * stride;
    }
    h.j = j;
    h.npar = 1 - par;
    h.mu = mu;
    h.fwd = fwd;
    h.wrap = wrap;
    h.lpar = fwd ? par : 1 - par;
    h.lsite = fwd ? i : j;
    return h;
}

// t[s] = U chi[s] (forward) or U^+ chi[s] (backward) for the 4 spins, times the
// boundary phase on a wrapped hop; identity path: t = chi
__device__ __forceinline__ void ptc_transport(const Geom &g, const void *gauge, size_t slab, const PathHop &h,
                                              const cpx<float> chi[12], cpx<float> t[12]) {
    if (h.mu < 0) {
#pragma unroll
        for (int k = 0; k < 12; ++k) t[k] = chi[k];
        return;
    }
    cpx<float> u[9];
    LinkIO<WL_F32, 18>::load((const char *)gauge + (size_t)(h.lpar * 4 + h.mu) * slab, h.lsite, u);
    cpx<float> z = {1.f, 0.f};
    if (h.wrap && ((g.phase_mask >> h.mu) & 1)) z = {(float)g.zr[h.mu], h.fwd ? (float)g.zi[h.mu] : -(float)g.zi[h.mu]};
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            cpx<float> acc = {0.f, 0.f};
#pragma unroll
            for (int k = 0; k < 3; ++k)
                acc = h.fwd ? cfma(u[3 * r + k], chi[3 * s + k], acc) : cjfma(u[3 * k + r], chi[3 * s + k], acc);
            t[3 * s + r] = cmul(z, acc);
        }
}

template <bool BF16W>
__device__ __forceinline__ float2 ptc_weight(const void *w, long idx) {
    if constexpr (BF16W) {
        const uint32_t v = ((const uint32_t *)w)[idx];
        return make_float2(bf16_to_f32((uint16_t)(v & 0xffffu)), bf16_to_f32((uint16_t)(v >> 16)));
    } else {
        return ((const float2 *)w)[idx];
    }
}

template <bool BF16W>
__global__ void __launch_bounds__(256) k_ptc_layer(const PtcArgs a) {
    // the 9 x cin spin matrices of this block's output channel, as FP32 in LDS
    __shared__ float2 wl[PTC_NPATH * PTC_MAXC * 16];
    const int o = blockIdx.z, par = blockIdx.y;
    const int nw = PTC_NPATH * a.cin * 16;
    for (int k = threadIdx.x; k < nw; k += blockDim.x) {
        const int q = k / (a.cin * 16), rem = k - q * a.cin * 16, b = rem >> 4, st = rem & 15;
        // spin matrix M[s][t] of (path q, input b): forward W_q^{ob}; adjoint (W_p^{bo})^+ with p the
        // reverse path, stored here already transposed and conjugated
        float2 e;
        if (a.adjoint) {
            const int s_ = st >> 2, t_ = st & 3;
            e = ptc_weight<BF16W>(a.w, ((long)(ptc_reverse(q) * a.cin + b) * a.cout + o) * 16 + 4 * t_ + s_);
            e.y = -e.y;
        } else {
            e = ptc_weight<BF16W>(a.w, ((long)(q * a.cout + o) * a.cin + b) * 16 + st);
        }
        wl[k] = e;
    }
    __syncthreads();
    const long pt = (long)blockIdx.x * blockDim.x + threadIdx.x;  // point (site, rhs)
    if (pt >= a.vh * a.nrhs) return;
    const int i = (int)(pt / a.nrhs), rhs = (int)(pt - (long)i * a.nrhs);
    int c[4];
    eo_coords(a.g, i, par, c);
    cpx<float> acc[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] = {0.f, 0.f};
    for (int q = 0; q < PTC_NPATH; ++q) {
        const PathHop h = ptc_hop(a.g, i, par, c, q);
        cpx<float> chi[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) chi[k] = {0.f, 0.f};
        for (int b = 0; b < a.cin; ++b) {
            cpx<float> v[12];
            SpinorIO<WL_F32>::load(a.in + (2 * (size_t)b + h.npar) * a.half, (long)h.j * a.nrhs + rhs, v);
            const float2 *m = &wl[(q * a.cin + b) * 16];
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const float2 e = m[4 * s + t];
                    const cpx<float> ms = {e.x, e.y};
#pragma unroll
                    for (int cc = 0; cc < 3; ++cc) chi[3 * s + cc] = cfma(ms, v[3 * t + cc], chi[3 * s + cc]);
                }
        }
        cpx<float> t[12];
        ptc_transport(a.g, a.gauge, a.slab_bytes, h, chi, t);
#pragma unroll
        for (int k = 0; k < 12; ++k) acc[k] = acc[k] + t[k];
    }
    SpinorIO<WL_F32>::store(a.out + (2 * (size_t)o + par) * a.half, pt, acc);
}

// One input channel fanned out to cout > 1 output channels: a block takes 64
// points (site, rhs); first its 256 threads compute the 8 one-hop transports of
// each point once (into LDS), then every (point, output channel) pair mixes the
// nine transported spinors with its own weights.  The per-channel kernel above
// would repeat every transport for each output channel.
constexpr int PTC_FAN_SITES = 64;

template <bool BF16W>
__global__ void __launch_bounds__(256) k_ptc_layer_fan(const PtcArgs a) {
    __shared__ float2 ts[8 * 12 * PTC_FAN_SITES];   // transported spinors [path-1][component][site]
    __shared__ float2 wl[PTC_NPATH * PTC_MAXC * 16];  // spin matrices [path][output channel][4x4]
    const int par = blockIdx.y;
    const int nw = PTC_NPATH * a.cout * 16;
    for (int k = threadIdx.x; k < nw; k += blockDim.x) {
        const int q = k / (a.cout * 16), rem = k - q * a.cout * 16, o = rem >> 4, st = rem & 15;
        float2 e;
        if (a.adjoint) {
            // (W_p^{0 o})^+ of the forward layer (1 -> cout here is its cout_f = 1, cin_f = cout)
            e = ptc_weight<BF16W>(a.w, ((long)ptc_reverse(q) * a.cout + o) * 16 + 4 * (st & 3) + (st >> 2));
            e.y = -e.y;
        } else {
            e = ptc_weight<BF16W>(a.w, ((long)q * a.cout + o) * 16 + st);
        }
        wl[k] = e;
    }
    const long base = (long)blockIdx.x * PTC_FAN_SITES;
    for (int task = threadIdx.x; task < 8 * PTC_FAN_SITES; task += blockDim.x) {
        const int sl = task % PTC_FAN_SITES, q = task / PTC_FAN_SITES + 1;
        const long pt = base + sl;
        cpx<float> t[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) t[k] = {0.f, 0.f};
        if (pt < a.vh * a.nrhs) {
            const int i = (int)(pt / a.nrhs), rhs = (int)(pt - (long)i * a.nrhs);
            int c[4];
            eo_coords(a.g, i, par, c);
            const PathHop h = ptc_hop(a.g, i, par, c, q);
            cpx<float> v[12];
            SpinorIO<WL_F32>::load(a.in + (size_t)h.npar * a.half, (long)h.j * a.nrhs + rhs, v);
            ptc_transport(a.g, a.gauge, a.slab_bytes, h, v, t);
        }
#pragma unroll
        for (int k = 0; k < 12; ++k) ts[((q - 1) * 12 + k) * PTC_FAN_SITES + sl] = make_float2(t[k].re, t[k].im);
    }
    __syncthreads();
    for (int task = threadIdx.x; task < a.cout * PTC_FAN_SITES; task += blockDim.x) {
        const int sl = task % PTC_FAN_SITES, o = task / PTC_FAN_SITES;
        const long pt = base + sl;
        if (pt >= a.vh * a.nrhs) continue;
        cpx<float> acc[12], v[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) acc[k] = {0.f, 0.f};
        SpinorIO<WL_F32>::load(a.in + (size_t)par * a.half, pt, v);  // identity path
        for (int q = 0; q < PTC_NPATH; ++q) {
            if (q > 0) {
#pragma unroll
                for (int k = 0; k < 12; ++k) {
                    const float2 f = ts[((q - 1) * 12 + k) * PTC_FAN_SITES + sl];
                    v[k] = {f.x, f.y};
                }
            }
            const float2 *m = &wl[(q * a.cout + o) * 16];
#pragma unroll
            for (int s_ = 0; s_ < 4; ++s_)
#pragma unroll
                for (int t_ = 0; t_ < 4; ++t_) {
                    const float2 e = m[4 * s_ + t_];
                    const cpx<float> ms = {e.x, e.y};
#pragma unroll
                    for (int cc = 0; cc < 3; ++cc) acc[3 * s_ + cc] = cfma(ms, v[3 * t_ + cc], acc[3 * s_ + cc]);
                }
        }
        SpinorIO<WL_F32>::store(a.out + (2 * (size_t)o + par) * a.half, pt, acc);
    }
}

// Two-pass form of a layer with one output channel and cin > 1 input channels
// (the 8 -> 1 layer and the adjoint of the 1 -> 8 layer).  The spin matrices act
// before the transports, so the mixing of path q, v_q(y) = sum_b M_q^b in_b(y),
// can be done at the source point y, once, for all the output points that reach
// y along q; then out(x) = sum_q T_q v_q(x + q) gathers nine single spinors.  The
// one-pass kernel above instead mixes the 8 input channels again at each of the
// nine neighbours (72 spinor loads per output point).  Pass 1: a thread per
// (point, group of 3 paths) reads the point's input channels once and keeps three
// mixtures; the per-point arithmetic is that of the one-pass kernel.
constexpr int PTC_MIX_GROUP = 3;
static_assert(PTC_NPATH % PTC_MIX_GROUP == 0, "paths split into whole groups");

template <bool BF16W>
__global__ void __launch_bounds__(256) k_ptc_mix(const PtcArgs a) {
    __shared__ float2 wl[PTC_MIX_GROUP * PTC_MAXC * 16];  // spin matrices [path in group][input][4x4]
    const int par = blockIdx.y, q0 = blockIdx.z * PTC_MIX_GROUP;
    const int nw = PTC_MIX_GROUP * a.cin * 16;
    for (int k = threadIdx.x; k < nw; k += blockDim.x) {
        const int g = k / (a.cin * 16), rem = k - g * a.cin * 16, b = rem >> 4, st = rem & 15;
        const int q = q0 + g;
        float2 e;
        if (a.adjoint) {
            const int s_ = st >> 2, t_ = st & 3;
            e = ptc_weight<BF16W>(a.w, ((long)(ptc_reverse(q) * a.cin + b) * a.cout + 0) * 16 + 4 * t_ + s_);
            e.y = -e.y;
        } else {
            e = ptc_weight<BF16W>(a.w, ((long)(q * a.cout + 0) * a.cin + b) * 16 + st);
        }
        wl[k] = e;
    }
    __syncthreads();
    const long pt = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (pt >= a.vh * a.nrhs) return;
    cpx<float> chi[PTC_MIX_GROUP][12];
#pragma unroll
    for (int g = 0; g < PTC_MIX_GROUP; ++g)
#pragma unroll
        for (int k = 0; k < 12; ++k) chi[g][k] = {0.f, 0.f};
    for (int b = 0; b < a.cin; ++b) {
        cpx<float> v[12];
        SpinorIO<WL_F32>::load(a.in + (2 * (size_t)b + par) * a.half, pt, v);
#pragma unroll
        for (int g = 0; g < PTC_MIX_GROUP; ++g) {
            const float2 *m = &wl[(g * a.cin + b) * 16];
#pragma unroll
            for (int s_ = 0; s_ < 4; ++s_)
#pragma unroll
                for (int t_ = 0; t_ < 4; ++t_) {
                    const float2 e = m[4 * s_ + t_];
                    const cpx<float> ms = {e.x, e.y};
#pragma unroll
                    for (int cc = 0; cc < 3; ++cc) chi[g][3 * s_ + cc] = cfma(ms, v[3 * t_ + cc], chi[g][3 * s_ + cc]);
                }
        }
    }
#pragma unroll
    for (int g = 0; g < PTC_MIX_GROUP; ++g)
        SpinorIO<WL_F32>::store(a.paths + (2 * (size_t)(q0 + g) + par) * a.half, pt, chi[g]);
}

// Pass 2: out(x) = sum_q T_q v_q(x + q), the nine mixtures of the neighbours
__global__ void __launch_bounds__(256) k_ptc_gather(const PtcArgs a) {
    const int par = blockIdx.y;
    const long pt = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (pt >= a.vh * a.nrhs) return;
    const int i = (int)(pt / a.nrhs), rhs = (int)(pt - (long)i * a.nrhs);
    int c[4];
    eo_coords(a.g, i, par, c);
    cpx<float> acc[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] = {0.f, 0.f};
    for (int q = 0; q < PTC_NPATH; ++q) {
        const PathHop h = ptc_hop(a.g, i, par, c, q);
        cpx<float> chi[12], t[12];
        SpinorIO<WL_F32>::load(a.paths + (2 * (size_t)q + h.npar) * a.half, (long)h.j * a.nrhs + rhs, chi);
        ptc_transport(a.g, a.gauge, a.slab_bytes, h, chi, t);
#pragma unroll
        for (int k = 0; k < 12; ++k) acc[k] = acc[k] + t[k];
    }
    SpinorIO<WL_F32>::store(a.out + (size_t)par * a.half, pt, acc);
}

hipError_t launch_ptc_layer(const PtcArgs &a, bool bf16, hipStream_t s) {
    if (a.cout < 1 || a.cin < 1 || a.cout * a.cin > PTC_MAXC || a.nrhs < 1) return hipErrorInvalidValue;
    const long npts = a.vh * a.nrhs;
    if (a.cin == 1 && a.cout > 1) {
        dim3 grid((unsigned)((npts + PTC_FAN_SITES - 1) / PTC_FAN_SITES), 2);
        if (bf16) hipLaunchKernelGGL(k_ptc_layer_fan<true>, grid, dim3(256), 0, s, a);
        else hipLaunchKernelGGL(k_ptc_layer_fan<false>, grid, dim3(256), 0, s, a);
        return hipGetLastError();
    }
    if (a.cout == 1 && a.cin > 1 && a.paths) {
        dim3 g1((unsigned)((npts + 255) / 256), 2, PTC_NPATH / PTC_MIX_GROUP);
        if (bf16) hipLaunchKernelGGL(k_ptc_mix<true>, g1, dim3(256), 0, s, a);
        else hipLaunchKernelGGL(k_ptc_mix<false>, g1, dim3(256), 0, s, a);
        hipLaunchKernelGGL(k_ptc_gather, dim3((unsigned)((npts + 255) / 256), 2), dim3(256), 0, s, a);
        return hipGetLastError();
    }
    dim3 grid((unsigned)((npts + 255) / 256), 2, (unsigned)a.cout);
    if (bf16) hipLaunchKernelGGL(k_ptc_layer<true>, grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL(k_ptc_layer<false>, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------- weight gradient
__global__ void __launch_bounds__(256) k_ptc_wgrad(const PtcGradArgs a) {
    const int combo = blockIdx.y;
    const int p = combo / (a.cout * a.cin);
    const int ab = combo - p * a.cout * a.cin;
    const int ao = ab / a.cin, b = ab - ao * a.cin;
    const long nsite = 2 * a.vh;
    const long per = (nsite + a.nchunks - 1) / a.nchunks;
    const long s0 = blockIdx.x * per, s1 = min(nsite, s0 + per);
    float gr[16], gi[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) gr[k] = gi[k] = 0.f;
    for (long x = s0 + threadIdx.x; x < s1; x += blockDim.x) {
        const int par = x >= a.vh ? 1 : 0;
        const int i = (int)(x - par * a.vh);
        int c[4];
        eo_coords(a.g, i, par, c);
        const PathHop h = ptc_hop(a.g, i, par, c, p);
        cpx<float> v[12], t[12], gg[12];
        SpinorIO<WL_F32>::load(a.in + (2 * (size_t)b + h.npar) * a.half, h.j, v);
        ptc_transport(a.g, a.gauge, a.slab_bytes, h, v, t);
        SpinorIO<WL_F32>::load(a.gout + (2 * (size_t)ao + par) * a.half, i, gg);
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int tt = 0; tt < 4; ++tt) {
                cpx<float> acc = {gr[4 * s + tt], gi[4 * s + tt]};
#pragma unroll
                for (int cc = 0; cc < 3; ++cc) acc = cjfma(t[3 * tt + cc], gg[3 * s + cc], acc);  // g conj(t)
                gr[4 * s + tt] = acc.re;
                gi[4 * s + tt] = acc.im;
            }
    }
    // block reduction of the 32 values (wavefront shuffles, then LDS)
    __shared__ float red[4][32];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        float r = gr[k], im = gi[k];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            r += __shfl_xor(r, off, 64);
            im += __shfl_xor(im, off, 64);
        }
        if (lane == 0) {
            red[wid][2 * k] = r;
            red[wid][2 * k + 1] = im;
        }
    }
    __syncthreads();
    if (threadIdx.x < 32) {
        float s = 0.f;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w][threadIdx.x];
        a.partials[((long)combo * a.nchunks + blockIdx.x) * 32 + threadIdx.x] = s;
    }
}

__global__ void __launch_bounds__(64) k_ptc_wgrad_reduce(const float *partials, int nchunks, double *grad,
                                                         int accumulate) {
    const int combo = blockIdx.x;
    if (threadIdx.x >= 32) return;
    double s = 0.0;
    for (int ch = 0; ch < nchunks; ++ch) s += (double)partials[((long)combo * nchunks + ch) * 32 + threadIdx.x];
    double *d = grad + (long)combo * 32 + threadIdx.x;
    *d = accumulate ? *d + s : s;
}

hipError_t launch_ptc_wgrad(const PtcGradArgs &a, double *grad, int accumulate, hipStream_t s) {
    const int ncombo = PTC_NPATH * a.cout * a.cin;
    if (a.cout < 1 || a.cin < 1 || a.nchunks < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_ptc_wgrad, dim3(a.nchunks, ncombo), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_ptc_wgrad_reduce, dim3(ncombo), dim3(64), 0, s, a.partials, a.nchunks, grad, accumulate);
    return hipGetLastError();
}

// ---------------------------------------------------------------- loss
__global__ void __launch_bounds__(256) k_ptc_loss(const void *out, const void *e, void *g, long n, const double *e2,
                                                  double inv_n, double *partials) {
    const int h = blockIdx.y;
    const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t hb = (size_t)padded(n) * 96;
    double d2 = 0.0;
    if (gid < n) {
        cpx<float> o[12], t[12];
        SpinorIO<WL_F32>::load((const char *)out + h * hb, gid, o);
        SpinorIO<WL_F32>::load((const char *)e + h * hb, gid, t);
        const float scale = (float)(inv_n / *e2);
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            const cpx<float> d = o[k] - t[k];
            d2 += (double)d.re * d.re + (double)d.im * d.im;
            o[k] = scale * d;
        }
        SpinorIO<WL_F32>::store((char *)g + h * hb, gid, o);
    }
    __shared__ double lds[16];
    const double s = block_sum(d2, lds);
    if (threadIdx.x == 0) partials[(long)blockIdx.y * gridDim.x + blockIdx.x] = s;
}

__global__ void __launch_bounds__(256) k_ptc_loss_reduce(const double *partials, long nblk, const double *e2,
                                                         double inv_n, double *loss) {
    __shared__ double lds[16];
    double s = 0.0;
    for (long b = threadIdx.x; b < nblk; b += blockDim.x) s += partials[b];
    s = block_sum(s, lds);
    if (threadIdx.x == 0) *loss += s * inv_n / *e2;
}

hipError_t launch_ptc_loss(const void *out, const void *e, void *g, long n, const double *e2, double inv_n,
                           double *partials, long stride, double *loss, hipStream_t s) {
    (void)stride;
    dim3 grid((unsigned)((n + 255) / 256), 2);
    hipLaunchKernelGGL(k_ptc_loss, grid, dim3(256), 0, s, out, e, g, n, e2, inv_n, partials);
    hipLaunchKernelGGL(k_ptc_loss_reduce, dim3(1), dim3(256), 0, s, partials, (long)grid.x * 2, e2, inv_n, loss);
    return hipGetLastError();
}

// ---------------------------------------------------------------- Adam
// omb1 = 1 - b1 and omb2 = 1 - b2 are formed in FP64 by the host: 1 - b2 computed in FP32 from the
// rounded b2 = 0.999f would be 1.3e-5 off (1 - 0.99900001f)
__global__ void __launch_bounds__(256) k_adam(float *w, uint16_t *wb, double *grad_c, float *m, float *v, long n,
                                              float lr, float b1, float b2, float omb1, float omb2, float eps,
                                              float c1, float c2) {
    const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    // grad_c holds (re, im) pairs of dL/dW*; the real-parameter gradient is twice that
    const float g = (float)(2.0 * grad_c[k]);
    grad_c[k] = 0.0;
    const float mk = b1 * m[k] + omb1 * g;
    const float vk = b2 * v[k] + omb2 * g * g;
    m[k] = mk;
    v[k] = vk;
    const float wk = w[k] - lr * (mk / c1) / (sqrtf(vk / c2) + eps);
    w[k] = wk;
    wb[k] = f32_to_bf16(wk);
}

hipError_t launch_adam(float *w, uint16_t *wb, double *grad_c, float *m, float *v, long n, double lr, double b1,
                       double b2, double eps, int t, hipStream_t s) {
    const float c1 = (float)(1.0 - std::pow(b1, (double)t)), c2 = (float)(1.0 - std::pow(b2, (double)t));
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, w, wb, grad_c, m, v, n, (float)lr,
                       (float)b1, (float)b2, (float)(1.0 - b1), (float)(1.0 - b2), (float)eps, c1, c2);
    return hipGetLastError();
}

__global__ void __launch_bounds__(256) k_to_bf16(const float *w, uint16_t *wb, long n) {
    const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) wb[k] = f32_to_bf16(w[k]);
}

hipError_t launch_to_bf16(const float *w, uint16_t *wb, long n, hipStream_t s) {
    hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, w, wb, n);
    return hipGetLastError();
}

}  // namespace wl
