// Launch interface of the hopping-term kernels.
#pragma once

#include "wl_common.h"

namespace wl {

enum : int { EPI_XPAY = 1, EPI_NORM = 2 };

struct HopArgs {
    Geom g;
    const void *in[2];    // input field of parity 0 / 1 (only the parity opposite to the output is read)
    void *out[2];         // output field of parity 0 / 1
    const void *x[2];     // epilogue field (same parity as the output), for EPI_XPAY
    const void *gauge;    // link storage: slabs (parity, mu), each `slab_bytes` long
    size_t slab_bytes;
    int out_par0;         // parity of blockIdx.y == 0
    int nrhs;
    long npts;            // points per parity = vh * nrhs
    double a, b;          // out = a x + b (H in)   (a ignored without EPI_XPAY)
    double *partials;     // EPI_NORM: per-block, per-rhs partial sums of ||out||^2
    long part_stride;     // distance between the partials of consecutive rhs
    const int *flag;      // if non-null and *flag != 0 the launch does nothing
    int swizzle;          // map consecutive blocks to the same XCD
};

struct LaunchCfg {
    int block = 256;
    int swizzle = 1;
};

// Enqueue out = a x + b H in (H^+ if dagger) over `nparity` output parities.
// Returns hipSuccess or the launch error.
hipError_t launch_hop(int prec, int recon, bool dagger, int epi, HopArgs &a, int nparity,
                      const LaunchCfg &cfg, hipStream_t stream);

// number of blocks per parity for a given configuration
inline long hop_blocks(long npts, int block) { return (npts + block - 1) / block; }

}  // namespace wl
