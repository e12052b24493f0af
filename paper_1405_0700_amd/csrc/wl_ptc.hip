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

// Pass 2: out(x) = sum_q T_q v_q(x + q), the nine mixtures of the neighbours.
// NT: the path fields are read with non-temporal loads (every value is read
// once; keeps them from evicting the links and the output from the caches).
template <bool NT>
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
        const char *base = a.paths + (2 * (size_t)q + h.npar) * a.half;
        if constexpr (NT) {
            const v4f *p = (const v4f *)base + blk_unit((long)h.j * a.nrhs + rhs, 6, 0);
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                const v4f d = __builtin_nontemporal_load(p + k * BLK);
                chi[2 * k] = {d[0], d[1]};
                chi[2 * k + 1] = {d[2], d[3]};
            }
        } else {
            SpinorIO<WL_F32>::load(base, (long)h.j * a.nrhs + rhs, chi);
        }
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
        hipLaunchKernelGGL(k_ptc_gather<false>, dim3((unsigned)((npts + 255) / 256), 2), dim3(256), 0, s, a);
        return hipGetLastError();
    }
    dim3 grid((unsigned)((npts + 255) / 256), 2, (unsigned)a.cout);
    if (bf16) hipLaunchKernelGGL(k_ptc_layer<true>, grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL(k_ptc_layer<false>, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------- network on matrix cores
// The network out = L2(L1(in)) is linear, and the spin matrices of a layer act
// before its transports, so the second layer's mixing of each path can be done
// at the source point (as in the two-pass form above): at every point y
//   t_q(y) = (T_q in)(y)                              nine transports
//   h_o(y) = sum_q W1_q^o t_q(y)                      first layer, C channels
//   v_p(y) = sum_o W2_p^o h_o(y)                      second layer, per path p
// and out(x) = sum_p T_p v_p(x + p) (k_ptc_gather).  The C-channel hidden field
// never leaves the registers.  Both mixings are real matrix products, each
// complex 4x4 spin matrix w = a + ib becoming the 8x8 real block with entries
// [re <- re] = a, [re <- im] = -b, [im <- re] = b, [im <- im] = a:
//   H (8C x 16) = A1 (8C x 96) T (96 x 16),  V (80 x 16) = A2 (80 x 8C) H,
// per colour, with 16 points (site, rhs) as the columns.  A wave takes 16 points
// and runs v_mfma_f32_16x16x32_bf16: the weights are BF16 already (exact); each
// FP32 activation is split exactly into three BF16 parts (hi = its top 16 bits,
// mid = the top 16 bits of the remainder, lo = the rest, at most 8 significant
// bits), so every product is exact and the sums are FP32 accumulations.
// MFMA lane layout (lane l, g = l / 16, n = l % 16): A row l % 16, columns
// 8 g .. 8 g + 7; B rows 8 g .. 8 g + 7, column n; D rows 4 g .. 4 g + 3,
// column n.  The K order inside a 32-column block is free (the same for A and
// B), so each lane feeds B with what it holds:
//   layer 1, K blocks 0 and 1: lane group g computes path 1 + 4 kb + g for point
//     n and supplies its 8 reals (spin, re / im) of one colour;
//   layer 1, K block 2: the identity path, its hi / mid / lo parts in lane groups
//     0 / 1 / 2 (A repeats the path-0 weights for each), group 3 zero;
//   layer 2, K block kb2: the lane's accumulators of layer-1 M tiles 2 kb2 and
//     2 kb2 + 1 (rows 4 g + i of each), three MFMAs for hi / mid / lo.
// Row orders: H row 8 o + 2 s + c (channel o, spin s, c = re / im); V row
// 8 p + 2 s + c, rows 72..79 zero.  A lane of a layer-2 output tile then holds
// spins 2 (g & 1), 2 (g & 1) + 1 of path 2 mt + g / 2 for one colour: with the
// three colours, three whole float4 units of the FP32 spinor layout.
typedef __bf16 ptc_bf16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t ptc_u32x4 __attribute__((ext_vector_type(4)));
typedef float ptc_f32x4 __attribute__((ext_vector_type(4)));

constexpr int PTC_NET_NM2 = 5;  // layer-2 M tiles (72 rows padded to 80)
__host__ __device__ constexpr int ptc_net_blocks(int C) { return 3 * (C / 2) + PTC_NET_NM2 * (C / 4); }

bool ptc_net_supported(int channels) { return channels == 4 || channels == 8; }
long ptc_net_table_elems(int channels) { return (long)ptc_net_blocks(channels) * 64 * 8; }

__device__ __forceinline__ ptc_f32x4 ptc_mfma(ptc_u32x4 a, ptc_u32x4 b, ptc_f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(ptc_bf16x8, a), __builtin_bit_cast(ptc_bf16x8, b),
                                                    c, 0, 0, 0);
}

// exact three-way BF16 split of two floats x0 (low half) and x1 (high half);
// v_perm_b32 with selector 0x07060302 packs the top 16 bits of two words
__device__ __forceinline__ uint32_t ptc_pack_hi(uint32_t lo_word, uint32_t hi_word) {
    return __builtin_amdgcn_perm(hi_word, lo_word, 0x07060302u);
}
__device__ __forceinline__ void ptc_split2(float x0, float x1, uint32_t &hi, uint32_t &mid, uint32_t &lo) {
    const uint32_t b0 = __float_as_uint(x0), b1 = __float_as_uint(x1);
    const float r0 = x0 - __uint_as_float(b0 & 0xffff0000u), r1 = x1 - __uint_as_float(b1 & 0xffff0000u);
    const uint32_t c0 = __float_as_uint(r0), c1 = __float_as_uint(r1);
    const float s0 = r0 - __uint_as_float(c0 & 0xffff0000u), s1 = r1 - __uint_as_float(c1 & 0xffff0000u);
    hi = ptc_pack_hi(b0, b1);
    mid = ptc_pack_hi(c0, c1);
    lo = ptc_pack_hi(__float_as_uint(s0), __float_as_uint(s1));
}

// the 8 reals (spin s = 0..3, re / im) of colour j, split into hi / mid / lo
__device__ __forceinline__ void ptc_split_colour(const cpx<float> v[12], int j, ptc_u32x4 out[3]) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        uint32_t h, m, l;
        ptc_split2(v[3 * s + j].re, v[3 * s + j].im, h, m, l);
        out[0][s] = h;
        out[1][s] = m;
        out[2][s] = l;
    }
}

// one part of the split of x, as a word whose top 16 bits are that part: with
// d1 = 1, d2 = 0 the mid part, with d1 = d2 = 1 the lo part, with both 0 the hi
// part (x itself); fma(-1, h, x) = x - h exactly, fma(-0, h, x) = x
__device__ __forceinline__ uint32_t ptc_part(float x, float d1, float d2) {
    const float r = fmaf(-d1, __uint_as_float(__float_as_uint(x) & 0xffff0000u), x);
    const float t = fmaf(-d2, __uint_as_float(__float_as_uint(r) & 0xffff0000u), r);
    return __float_as_uint(t);
}

// Operand tables: block b < 3 C / 2 is layer-1 (M tile b / 3, K block b % 3),
// then layer-2 (M tile, K block) = ((b - 3 C / 2) / (C / 4), (b - 3 C / 2) % (C / 4));
// each block is [lane][8] BF16, lane l holding its A fragment.  Forward: layer 1
// W1_q^{o}, layer 2 W2_p^{o}.  Adjoint: layer 1 (W2_{rev q}^{o})^+, layer 2
// (W1_{rev p}^{o})^+ (the transports of M^+ run along the reversed paths).
template <int C>
__global__ void __launch_bounds__(256) k_ptc_net_table(const uint16_t *wb, long n1, uint16_t *tab, int adjoint) {
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)ptc_net_blocks(C) * 512) return;
    const int i = (int)(idx & 7), l = (int)((idx >> 3) & 63), blk = (int)(idx >> 9);
    const int g = l >> 4;
    const uint16_t *w1 = wb, *w2 = wb + 2 * n1;
    int row_o, row_s, row_c, q, t, col_c;  // output (channel or path, spin, re/im), input (path or channel, spin, re/im)
    bool zero = false, layer1 = blk < 3 * (C / 2);
    if (layer1) {
        const int mt = blk / 3, kb = blk % 3, m = 16 * mt + (l & 15);
        row_o = m >> 3; row_s = (m & 7) >> 1; row_c = m & 1;
        q = kb < 2 ? 1 + 4 * kb + g : 0;
        zero = kb == 2 && g == 3;
        t = i >> 1; col_c = i & 1;
    } else {
        const int b2 = blk - 3 * (C / 2), mt2 = b2 / (C / 4), kb2 = b2 % (C / 4), r = 16 * mt2 + (l & 15);
        zero = r >= 8 * PTC_NPATH;
        row_o = r >> 3; row_s = (r & 7) >> 1; row_c = r & 1;
        const int h = 32 * kb2 + (i < 4 ? 4 * g + i : 16 + 4 * g + (i - 4));
        q = h >> 3; t = (h & 7) >> 1; col_c = h & 1;  // q: hidden channel here
    }
    uint16_t v = 0;
    if (!zero) {
        // complex weight (re, im) as BF16 bits
        long cidx;
        const uint16_t *base;
        bool conj = false;
        if (layer1) {
            // row_o: channel o, q: path
            if (!adjoint) { base = w1; cidx = ((long)q * C + row_o) * 16 + 4 * row_s + t; }
            else { base = w2; cidx = ((long)ptc_reverse(q) * C + row_o) * 16 + 4 * t + row_s; conj = true; }
        } else {
            // row_o: path p, q: channel o
            if (!adjoint) { base = w2; cidx = ((long)row_o * C + q) * 16 + 4 * row_s + t; }
            else { base = w1; cidx = ((long)ptc_reverse(row_o) * C + q) * 16 + 4 * t + row_s; conj = true; }
        }
        const uint16_t re = base[2 * cidx];
        const uint16_t im = conj ? (uint16_t)(base[2 * cidx + 1] ^ 0x8000u) : base[2 * cidx + 1];
        // [re <- re] = a, [re <- im] = -b, [im <- re] = b, [im <- im] = a
        v = row_c == 0 ? (col_c == 0 ? re : (uint16_t)(im ^ 0x8000u)) : (col_c == 0 ? im : re);
    }
    tab[idx] = v;
}

hipError_t launch_ptc_net_tables(const uint16_t *wb, long n1, int channels, uint16_t *tab_fwd, uint16_t *tab_adj,
                                 hipStream_t s) {
    if (!ptc_net_supported(channels)) return hipErrorInvalidValue;
    const long n = ptc_net_table_elems(channels);
    const unsigned blocks = (unsigned)((n + 255) / 256);
    for (int adj = 0; adj < 2; ++adj) {
        uint16_t *tab = adj ? tab_adj : tab_fwd;
        if (channels == 8) hipLaunchKernelGGL(k_ptc_net_table<8>, dim3(blocks), dim3(256), 0, s, wb, n1, tab, adj);
        else hipLaunchKernelGGL(k_ptc_net_table<4>, dim3(blocks), dim3(256), 0, s, wb, n1, tab, adj);
    }
    return hipGetLastError();
}

// t = U chi (forward hop) or U^+ chi (backward hop) for the 4 spins, times the
// boundary phase on a wrapped hop, without branching on the direction: the
// lanes of a wave take different paths, so the backward link is transposed and
// conjugated by selects and one multiply sequence serves both; the phase
// multiply is skipped when no lane of the wave wraps.  Hop paths only (q >= 1).
__device__ __forceinline__ void ptc_transport_sel(const Geom &g, const void *gauge, size_t slab, const PathHop &h,
                                                  bool active, const cpx<float> chi[12], cpx<float> t[12]) {
    cpx<float> u[9];
    LinkIO<WL_F32, 18>::load((const char *)gauge + (size_t)(h.lpar * 4 + h.mu) * slab, h.lsite, u);
    cpx<float> m[9];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const cpx<float> a = u[3 * r + k], b = u[3 * k + r];
            m[3 * r + k] = h.fwd ? a : cpx<float>{b.re, -b.im};
        }
    const bool wraps = active && h.wrap && ((g.phase_mask >> h.mu) & 1);
    if (__builtin_amdgcn_ballot_w64(wraps)) {
        const cpx<float> z = wraps ? cpx<float>{(float)g.zr[h.mu], h.fwd ? (float)g.zi[h.mu] : -(float)g.zi[h.mu]}
                                   : cpx<float>{1.f, 0.f};
#pragma unroll
        for (int k = 0; k < 9; ++k) m[k] = cmul(z, m[k]);
    }
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            cpx<float> acc = {0.f, 0.f};
#pragma unroll
            for (int k = 0; k < 3; ++k) acc = cfma(m[3 * r + k], chi[3 * s + k], acc);
            t[3 * s + r] = acc;
        }
}

// Pass A; a wave per tile of 16 points of one parity, tiles of both parities in
// one range (parity = tile / tiles_per_parity), waves loop over tiles.
template <int C>
__global__ void __launch_bounds__(256, 2) k_ptc_net_mix(const PtcArgs a, const uint16_t *tab, long tiles_par) {
    constexpr int NM1 = C / 2, NK2 = C / 4, NB = ptc_net_blocks(C);
    __shared__ ptc_u32x4 ta[NB * 64];
    for (int k = threadIdx.x; k < NB * 64; k += blockDim.x) ta[k] = ((const ptc_u32x4 *)tab)[k];
    __syncthreads();
    const int lane = threadIdx.x & 63, g = lane >> 4, n = lane & 15;
    const long npts = a.vh * a.nrhs;
    const long ntile = 2 * tiles_par;
    for (long tile = (long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); tile < ntile;
         tile += (long)gridDim.x * (blockDim.x >> 6)) {
        const int par = tile >= tiles_par ? 1 : 0;
        const long pt = (tile - par * tiles_par) * 16 + n;
        const bool valid = pt < npts;
        int i = 0, rhs = 0;
        int c[4] = {0, 0, 0, 0};
        if (valid) {
            // npts < 2^31 (checked at launch)
            i = (int)pt / a.nrhs;
            rhs = (int)pt - i * a.nrhs;
            eo_coords(a.g, i, par, c);
        }
        ptc_f32x4 acc1[NM1][3];
#pragma unroll
        for (int mt = 0; mt < NM1; ++mt)
#pragma unroll
            for (int j = 0; j < 3; ++j) acc1[mt][j] = ptc_f32x4{0.f, 0.f, 0.f, 0.f};
        // layer 1, hop paths: K blocks 0 and 1
#pragma unroll 1
        for (int kb = 0; kb < 2; ++kb) {
            // invalid points (the last tile's tail) take site 0 with zero input and store nothing
            const PathHop h = ptc_hop(a.g, i, par, c, 1 + 4 * kb + g);
            cpx<float> v[12];
            if (valid) {
                SpinorIO<WL_F32>::load(a.in + (size_t)h.npar * a.half, (long)h.j * a.nrhs + rhs, v);
            } else {
#pragma unroll
                for (int k = 0; k < 12; ++k) v[k] = {0.f, 0.f};
            }
            cpx<float> t[12];
            ptc_transport_sel(a.g, a.gauge, a.slab_bytes, h, valid, v, t);
            ptc_u32x4 b[3][3];
#pragma unroll
            for (int j = 0; j < 3; ++j) ptc_split_colour(t, j, b[j]);
#pragma unroll
            for (int mt = 0; mt < NM1; ++mt) {
                const ptc_u32x4 w = ta[(mt * 3 + kb) * 64 + lane];
#pragma unroll
                for (int j = 0; j < 3; ++j)
#pragma unroll
                    for (int part = 2; part >= 0; --part) acc1[mt][j] = ptc_mfma(w, b[j][part], acc1[mt][j]);
            }
        }
        // layer 1, identity path: K block 2 (hi / mid / lo in lane groups 0 / 1 / 2)
        {
            cpx<float> v[12];
#pragma unroll
            for (int k = 0; k < 12; ++k) v[k] = {0.f, 0.f};
            if (valid && g < 3) SpinorIO<WL_F32>::load(a.in + (size_t)par * a.half, pt, v);
            ptc_u32x4 b[3];  // group 3 holds zeros (v = 0 there)
            const float d1 = g >= 1 ? 1.f : 0.f, d2 = g >= 2 ? 1.f : 0.f;
#pragma unroll
            for (int j = 0; j < 3; ++j)
#pragma unroll
                for (int s_ = 0; s_ < 4; ++s_)
                    b[j][s_] = ptc_pack_hi(ptc_part(v[3 * s_ + j].re, d1, d2), ptc_part(v[3 * s_ + j].im, d1, d2));
#pragma unroll
            for (int mt = 0; mt < NM1; ++mt) {
                const ptc_u32x4 w = ta[(mt * 3 + 2) * 64 + lane];
#pragma unroll
                for (int j = 0; j < 3; ++j) acc1[mt][j] = ptc_mfma(w, b[j], acc1[mt][j]);
            }
        }
        // layer 2
        ptc_u32x4 b2[NK2][3][3];
#pragma unroll
        for (int kb2 = 0; kb2 < NK2; ++kb2)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const ptc_f32x4 lo4 = acc1[2 * kb2][j], hi4 = acc1[2 * kb2 + 1][j];
                uint32_t h, m, l;
                ptc_split2(lo4[0], lo4[1], h, m, l);
                b2[kb2][j][0][0] = h; b2[kb2][j][1][0] = m; b2[kb2][j][2][0] = l;
                ptc_split2(lo4[2], lo4[3], h, m, l);
                b2[kb2][j][0][1] = h; b2[kb2][j][1][1] = m; b2[kb2][j][2][1] = l;
                ptc_split2(hi4[0], hi4[1], h, m, l);
                b2[kb2][j][0][2] = h; b2[kb2][j][1][2] = m; b2[kb2][j][2][2] = l;
                ptc_split2(hi4[2], hi4[3], h, m, l);
                b2[kb2][j][0][3] = h; b2[kb2][j][1][3] = m; b2[kb2][j][2][3] = l;
            }
#pragma unroll
        for (int mt2 = 0; mt2 < PTC_NET_NM2; ++mt2) {
            ptc_f32x4 acc[3];
#pragma unroll
            for (int j = 0; j < 3; ++j) acc[j] = ptc_f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kb2 = 0; kb2 < NK2; ++kb2) {
                const ptc_u32x4 w = ta[(3 * NM1 + mt2 * NK2 + kb2) * 64 + lane];
#pragma unroll
                for (int j = 0; j < 3; ++j)
#pragma unroll
                    for (int part = 2; part >= 0; --part) acc[j] = ptc_mfma(w, b2[kb2][j][part], acc[j]);
            }
            const int p = 2 * mt2 + (g >> 1);
            if (valid && p < PTC_NPATH) {
                // spins s0 = 2 (g & 1) and s0 + 1, colours 0..2: complex components 3 s0 .. 3 s0 + 5,
                // float4 units 3 (g & 1) .. 3 (g & 1) + 2
                // non-temporal: each path value is read once, by the gather
                v4f *dst = (v4f *)(a.paths + (2 * (size_t)p + par) * a.half) + blk_unit(pt, 6, 3 * (g & 1));
                st_out<true, v4f>(dst, v4f{acc[0][0], acc[0][1], acc[1][0], acc[1][1]});
                st_out<true, v4f>(dst + BLK, v4f{acc[2][0], acc[2][1], acc[0][2], acc[0][3]});
                st_out<true, v4f>(dst + 2 * BLK, v4f{acc[1][2], acc[1][3], acc[2][2], acc[2][3]});
            }
        }
    }
}

hipError_t launch_ptc_net(const PtcArgs &a, int channels, const uint16_t *tab, hipStream_t s) {
    if (!ptc_net_supported(channels) || !a.paths || a.nrhs < 1 || !tab) return hipErrorInvalidValue;
    const long npts = a.vh * a.nrhs;
    if (npts + 16 > INT_MAX) return hipErrorInvalidValue;
    const long tiles_par = (npts + 15) / 16;
    const long waves = 2 * tiles_par;
    const unsigned blocks = (unsigned)std::min<long>((waves + 3) / 4, 2048);
    if (channels == 8) hipLaunchKernelGGL(k_ptc_net_mix<8>, dim3(blocks), dim3(256), 0, s, a, tab, tiles_par);
    else hipLaunchKernelGGL(k_ptc_net_mix<4>, dim3(blocks), dim3(256), 0, s, a, tab, tiles_par);
    hipLaunchKernelGGL(k_ptc_gather<true>, dim3((unsigned)((npts + 255) / 256), 2), dim3(256), 0, s, a);
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
