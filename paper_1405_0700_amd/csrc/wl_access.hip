// Link-spinor access kernels: psi(x_i) = U(x_i) phi(x_i), the colour matrix of a
// site applied to the four colour vectors of its spinor, with the site sequence
// x_i taken in order, through an index array, or through precomputed addresses
// (the paper's isolated link-spinor kernel of its section on overlapping
// communication with computation, and its comparison of addressing schemes).
//
// One thread per step i; every component is a 16-byte FP64 complex number.
// Layout 0 keeps a site's components together (U: 9, spinor: 12); layout 1 keeps
// blocks of 64 sites with component k of the block's sites side by side, the
// layout of the library's fields.
#include "wl_access.h"

namespace wl {

template <int NC, int LAYOUT>
__device__ __forceinline__ long site_base(long x) {
    if constexpr (LAYOUT == 0) return x * NC;
    else return (x >> 6) * 64 * NC + (x & 63);
}

template <int MODE, int LAYOUT>
__global__ void __launch_bounds__(256) k_su3_apply(const AccessArgs a) {
    constexpr long CS = LAYOUT == 0 ? 1 : 64;  // component stride in complex numbers
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    double2 *pp;
    const double2 *up, *fp;
    if constexpr (MODE == 2) {
        pp = (double2 *)a.ptrs[3 * i];
        up = (const double2 *)a.ptrs[3 * i + 1];
        fp = (const double2 *)a.ptrs[3 * i + 2];
    } else {
        const long x = MODE == 0 ? i : (long)a.index[i];
        pp = a.psi + site_base<12, LAYOUT>(x);
        up = a.u + site_base<9, LAYOUT>(x);
        fp = a.phi + site_base<12, LAYOUT>(x);
    }
    double2 u[9], f[12];
#pragma unroll
    for (int k = 0; k < 9; ++k) u[k] = up[k * CS];
#pragma unroll
    for (int k = 0; k < 12; ++k) f[k] = fp[k * CS];
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            double re = 0.0, im = 0.0;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const double2 m = u[3 * r + c], v = f[3 * s + c];
                re = fma(m.x, v.x, fma(-m.y, v.y, re));
                im = fma(m.x, v.y, fma(m.y, v.x, im));
            }
            pp[(3 * s + r) * CS] = make_double2(re, im);
        }
}

hipError_t launch_su3_apply(const AccessArgs &a, int mode, int layout, hipStream_t s) {
    if (a.n <= 0) return hipSuccess;
    const dim3 grid((unsigned)((a.n + 255) / 256)), block(256);
    switch (mode * 2 + layout) {
    case 0: hipLaunchKernelGGL((k_su3_apply<0, 0>), grid, block, 0, s, a); break;
    case 1: hipLaunchKernelGGL((k_su3_apply<0, 1>), grid, block, 0, s, a); break;
    case 2: hipLaunchKernelGGL((k_su3_apply<1, 0>), grid, block, 0, s, a); break;
    case 3: hipLaunchKernelGGL((k_su3_apply<1, 1>), grid, block, 0, s, a); break;
    case 4: hipLaunchKernelGGL((k_su3_apply<2, 0>), grid, block, 0, s, a); break;
    case 5: hipLaunchKernelGGL((k_su3_apply<2, 1>), grid, block, 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace wl
