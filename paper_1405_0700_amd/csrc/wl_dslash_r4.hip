// Instances of the hopping-term kernel that computes 4 right-hand sides per
// thread (each link load applied to all of them).
#include "wl_dslash_kernels.h"

namespace wl {
hipError_t launch_hop_r4(int prec, int recon, bool dag, bool nt, int epi, const HopArgs &a, dim3 grid, dim3 blk,
                         hipStream_t s) {
    return launch_hop_r_impl<4>(prec, recon, dag, nt, epi, a, grid, blk, s);
}
}  // namespace wl
