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
    const int *flag;      // if non-null and *flag == 0 (no system still iterating) the launch does nothing
    int swizzle;          // map consecutive blocks to the same XCD
    int tchunk;           // processing order (see LaunchCfg)
    int chunk_sites;      // sites of a full chunk: tchunk * Lz * (Lx/2) * Ly
};

struct LaunchCfg {
    int block = 256;   // threads per block (multiple of 64, <= 256)
    int swizzle = 1;   // give each XCD one contiguous range of blocks
    int tps = 1;       // threads per output point: 1, or 2 (forward / backward hops in
                       // the two halves of a wavefront; FP64 and FP32 storage only)
    int tchunk = 0;    // processing order: 0 = e/o index order; k = chunks of k time
                       // slices, each walked with z slowest
    int nt = -1;       // non-temporal link loads / output stores: 1 on, 0 off,
                       // -1 on when the launch's working set exceeds 200 MB
};

// whether a launch uses the non-temporal hints
bool use_nontemporal(int prec, const LaunchCfg &cfg, const HopArgs &a, int nparity, int epi);

// Enqueue out = a x + b H in (H^+ if dagger) over `nparity` output parities.
// Returns hipSuccess or the launch error.
hipError_t launch_hop(int prec, int recon, bool dagger, int epi, HopArgs &a, int nparity,
                      const LaunchCfg &cfg, hipStream_t stream);

// threads per point actually used for a storage precision
int effective_tps(int prec, const LaunchCfg &cfg);

// number of blocks per parity for a given configuration
inline long hop_blocks(long npts, int block, int tps = 1) { return (npts * tps + block - 1) / block; }

}  // namespace wl
