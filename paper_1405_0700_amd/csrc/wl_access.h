// Link-spinor access kernels (psi(x_i) = U(x_i) phi(x_i), FP64, three addressing
// modes, two layouts); the C entry point wl_su3_apply validates the arguments.
#pragma once

#include "wl_common.h"

namespace wl {

struct AccessArgs {
    double2 *psi;
    const double2 *u;
    const double2 *phi;
    long n;
    const int *index;               // mode 1: site of step i
    const unsigned long long *ptrs; // mode 2: psi, U, phi address of step i at 3 i .. 3 i + 2
};

// mode 0: x_i = i; 1: x_i = index[i]; 2: precomputed addresses.  layout 0: a site's
// components together; 1: blocks of 64 sites, component-major within a block.
hipError_t launch_su3_apply(const AccessArgs &a, int mode, int layout, hipStream_t s);

}  // namespace wl
