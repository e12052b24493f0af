// Launch interface of the hopping-term kernels.
#pragma once

#include "wl_common.h"

namespace wl {

// EPI_CGR (always with EPI_XPAY | EPI_NORM): the result y = a x + b H in is not
// stored; instead the CG residual r -= alpha y is updated in place (alpha of the
// point's rhs from the solver's device scalars; nothing happens where alpha = 0)
// and ||r||^2 is reduced.  One-point-per-thread kernels only (rpt = 1).
enum : int { EPI_XPAY = 1, EPI_NORM = 2, EPI_CGR = 4 };
// With non-temporal link loads (the kernels' NT), store the output through the
// caches all the same: set by the launcher for outputs small enough to be read
// again from the Infinity Cache by the next kernel of a solve.
enum : int { EPI_CACHED_OUT = 16 };

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
    double tm_x, tm_h;    // twists: x -> (1 + i tm_x gamma_5) x, H in -> (1 + i tm_h gamma_5) H in (0: none)
    double *partials;     // EPI_NORM: per-block, per-rhs partial sums of ||out||^2
    long part_stride;     // distance between the partials of consecutive rhs
    const int *flag;      // if non-null and *flag == 0 (no system still iterating) the launch does nothing
    int swizzle;          // map consecutive blocks to the same XCD
    int tchunk;           // processing order (see LaunchCfg)
    int chunk_sites;      // sites of a full chunk: tchunk * Lz * (Lx/2) * Ly
    int yz_by, yz_bz;     // WL_TCHUNK_YZ: block extent in y and z
    FastDiv f_blk, f_slab, f_row;  // WL_TCHUNK_YZ: sites of a block, of one of its t, of one of its (z, t)
    FastDiv f_chunk, f_kplane;     // z-ranges (tchunk < 0): chunk_sites, and -tchunk planes of (Lx/2) Ly sites
    void *r[2];           // EPI_CGR: the residual field of parity 0 / 1 (same storage as out)
    const char *alpha;    // EPI_CGR: alpha of rhs k at alpha + k * alpha_stride (a double)
    long alpha_stride;
    unsigned shm;         // dynamic LDS bytes reserved per block (host side: caps the occupancy)
    int sweep;            // time sweep: slices per block (0: one point per thread, no sweep)
};

// Site of position ps in the y-z block order (WL_TCHUNK_YZ): the (y, z) plane
// is cut into 2 x 4 blocks of by x bz x-lines; block b holds y in
// [(b % 2) by, +by) and z in [(b / 2) bz, +bz); its sites follow each other with
// t slowest, then z, y and x.  Returns the e/o index x + (Lx/2) y + sz z + st t.
__host__ __device__ __forceinline__ int yz_site(const Geom &g, int by, int bz, const FastDiv &f_blk,
                                                const FastDiv &f_slab, const FastDiv &f_row, int ps) {
    const int b = fdiv(ps, f_blk);
    const int r = ps - b * f_blk.d;
    const int t = fdiv(r, f_slab);
    const int q = r - t * f_slab.d;
    const int zl = fdiv(q, f_row);
    const int q2 = q - zl * f_row.d;
    const int yl = fdiv(q2, g.f_lxh);
    const int x = q2 - yl * g.lxh;
    return x + g.lxh * ((b & 1) * by + yl) + g.sz * ((b >> 1) * bz + zl) + g.st * t;
}

struct LaunchCfg {
    int block = 256;   // threads per block (multiple of 64, <= 256)
    int swizzle = 1;   // give each XCD one contiguous range of blocks
    int tps = 1;       // threads per output point: 1, or 2 (forward / backward hops in
                       // the two halves of a wavefront)
    int tchunk = WL_TCHUNK_AUTO;  // processing order: 0 = e/o index order; k > 0 = chunks of k
                       // time slices, each walked with z slowest; k < 0 = chunks of -k
                       // z-planes over all t, each walked with t slowest; WL_TCHUNK_YZ =
                       // 2 x 4 y-z blocks, each walked with t slowest; AUTO: -(Lz/8) when
                       // Lz is a multiple of 8 and >= 16, else 0
    int nt = -1;       // non-temporal link loads / output stores: 1 on, 0 off,
                       // -1 on when the launch's working set exceeds 200 MB
    int rpt = 1;       // right-hand sides per thread (each link load reused for all
                       // of them); used when nrhs % rpt == 0 and tps == 1
    int sweep = 0;     // k > 0: time sweep, each thread walks k slices of one point's column
                       // (its time neighbours kept in registers); used when tps == 1 and
                       // rpt == 1; 0: off
    int occ = 0;       // 0: no cap; k in 1..8: about k waves per SIMD at most (unused LDS is
                       // reserved per block, so that fewer blocks fit on a CU; fewer
                       // points in flight keep the re-read neighbours of multi-rhs
                       // launches within L2)
};

// dynamic LDS bytes per block that cap a launch of `block` threads at `occ`
// waves per SIMD (160 KB of LDS per CU, 4 SIMDs); 0 for no cap
unsigned occupancy_lds(int occ, int block, unsigned static_lds);

// whether a launch uses the non-temporal hints
bool use_nontemporal(int prec, const LaunchCfg &cfg, const HopArgs &a, int nparity, int epi);
// a.tchunk / a.chunk_sites for a LaunchCfg tchunk value (WL_TCHUNK_AUTO resolved from the lattice)
void set_processing_order(HopArgs &a, int tchunk);

// Enqueue out = a x + b H in (H^+ if dagger) over `nparity` output parities.
// Returns hipSuccess or the launch error.  ev0 / ev1, when given, time the
// launch: the kernel's own dispatch packet stamps its start and end (the
// one-point-per-thread, two-threads-per-point and sweep kernels), so that the
// interval is the kernel's execution, as a kernel trace reports it; the kernels
// with several right-hand sides per thread record them before and after.
hipError_t launch_hop(int prec, int recon, bool dagger, int epi, HopArgs &a, int nparity,
                      const LaunchCfg &cfg, hipStream_t stream, hipEvent_t ev0 = nullptr,
                      hipEvent_t ev1 = nullptr);

// Persistent launch over the tiles of several systems (one-thread-per-point
// body).  sys[k] is filled like a single launch's HopArgs (out_par0 = first
// output parity); tiles of system k: per_par[k] blocks of `block` points per
// output parity, np[k] parities; start[k] = first tile of system k in the
// concatenated list, start[nsys] = ntiles.
constexpr int BATCH_MAX = 8;
struct BatchArgs {
    HopArgs sys[BATCH_MAX];
    long start[BATCH_MAX + 1];
    long per_par[BATCH_MAX];
    int nsys;
    long ntiles;
};
// nwg: persistent workgroups (a multiple of 8); epi without EPI_NORM alone; tps 2
// (two threads per point, FP64/FP32 storage only): a tile holds block / 2 points
hipError_t launch_hop_batch(int prec, int recon, bool dagger, int epi, bool nt, int tps, BatchArgs &B, int nwg,
                            int block, hipStream_t stream);

// threads per point actually used for a storage precision
int effective_tps(int prec, const LaunchCfg &cfg);

// number of blocks per parity for a given configuration
inline long hop_blocks(long npts, int block, int tps = 1) { return (npts * tps + block - 1) / block; }

// right-hand sides per thread a launch of nrhs right-hand sides actually uses
inline int effective_rpt(const LaunchCfg &cfg, int nrhs, int tps) {
    return cfg.rpt > 1 && tps == 1 && nrhs % cfg.rpt == 0 ? cfg.rpt : 1;
}

// slices per block of a time-sweep launch (0: no sweep), for a lattice of lt time slices
inline int effective_sweep(const LaunchCfg &cfg, int nrhs, int tps, int lt, int prec = 0) {
    // 16-bit storage: the decode's multiply would contract differently with a spinor held
    // in registers than straight after its load, so the sweep is offered for FP64 / FP32 only
    if (cfg.sweep <= 0 || tps != 1 || effective_rpt(cfg, nrhs, tps) != 1 || prec > 1) return 0;
    return cfg.sweep < lt ? cfg.sweep : lt;
}

// blocks per parity of a hopping launch (npts points of nrhs right-hand sides; lt time
// slices, sites_per_slice sites of one parity per slice)
inline long hop_launch_blocks(int tps, const LaunchCfg &cfg, long npts, int nrhs, int lt = 0,
                              long sites_per_slice = 0, int prec = 0) {
    const int r = effective_rpt(cfg, nrhs, tps);
    if (const int sw = lt > 0 ? effective_sweep(cfg, nrhs, tps, lt, prec) : 0)
        return hop_blocks(sites_per_slice * nrhs, cfg.block, 1) * ((lt + sw - 1) / sw);
    return r > 1 ? hop_blocks(npts / r, cfg.block, 1) : hop_blocks(npts, cfg.block, tps);
}

}  // namespace wl
