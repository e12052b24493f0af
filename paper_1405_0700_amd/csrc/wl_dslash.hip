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
#include <algorithm>

#include <hip/hip_ext.h>

#include "wl_dslash_kernels.h"

namespace wl {

// Timing events of the launch being enqueued by this host thread (see launch_hop)
static thread_local hipEvent_t t_ev[2] = {nullptr, nullptr};

template <typename K> static void enqueue(K kern, dim3 grid, dim3 block, hipStream_t s, const HopArgs &a) {
    if (t_ev[0])
        hipExtLaunchKernelGGL(kern, grid, block, a.shm, s, t_ev[0], t_ev[1], 0, a);
    else
        hipLaunchKernelGGL(kern, grid, block, a.shm, s, a);
}

template <int SP, int GP, int RECON, bool DAG, int EPI, bool NT>
static void launch_one(int tps, dim3 grid, dim3 block, hipStream_t s, const HopArgs &a) {
    if (a.sweep > 0)
        enqueue(hop_sweep_kernel<SP, GP, RECON, DAG, EPI, NT>, grid, block, s, a);
    else if (tps == 2)
        enqueue(hop_kernel_split<SP, GP, RECON, DAG, EPI, NT>, grid, block, s, a);
    else
        enqueue(hop_kernel<SP, GP, RECON, DAG, EPI, NT>, grid, block, s, a);
}

template <int SP, int GP, int RECON, bool DAG, bool NT>
static hipError_t launch_epi(int epi, int tps, HopArgs &a, dim3 grid, dim3 block, hipStream_t s) {
    switch (epi) {
    case 0: launch_one<SP, GP, RECON, DAG, 0, NT>(tps, grid, block, s, a); break;
    case EPI_XPAY: launch_one<SP, GP, RECON, DAG, EPI_XPAY, NT>(tps, grid, block, s, a); break;
    case EPI_NORM: launch_one<SP, GP, RECON, DAG, EPI_NORM, NT>(tps, grid, block, s, a); break;
    case EPI_XPAY | EPI_NORM:
        launch_one<SP, GP, RECON, DAG, EPI_XPAY | EPI_NORM, NT>(tps, grid, block, s, a);
        break;
    case EPI_XPAY | EPI_NORM | EPI_CGR:
        launch_one<SP, GP, RECON, DAG, EPI_XPAY | EPI_NORM | EPI_CGR, NT>(tps, grid, block, s, a);
        break;
    default:
        if constexpr (NT) {
            constexpr int C = EPI_CACHED_OUT;
            switch (epi) {
            case C: launch_one<SP, GP, RECON, DAG, C, NT>(tps, grid, block, s, a); break;
            case C | EPI_XPAY: launch_one<SP, GP, RECON, DAG, C | EPI_XPAY, NT>(tps, grid, block, s, a); break;
            case C | EPI_NORM: launch_one<SP, GP, RECON, DAG, C | EPI_NORM, NT>(tps, grid, block, s, a); break;
            case C | EPI_XPAY | EPI_NORM:
                launch_one<SP, GP, RECON, DAG, C | EPI_XPAY | EPI_NORM, NT>(tps, grid, block, s, a);
                break;
            default: return hipErrorInvalidValue;
            }
            break;
        }
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int SP, int GP, int RECON>
static hipError_t launch_dag(bool dag, bool nt, int epi, int tps, HopArgs &a, dim3 grid, dim3 block,
                             hipStream_t s) {
    if (nt)
        return dag ? launch_epi<SP, GP, RECON, true, true>(epi, tps, a, grid, block, s)
                   : launch_epi<SP, GP, RECON, false, true>(epi, tps, a, grid, block, s);
    return dag ? launch_epi<SP, GP, RECON, true, false>(epi, tps, a, grid, block, s)
               : launch_epi<SP, GP, RECON, false, false>(epi, tps, a, grid, block, s);
}

bool use_nontemporal(int prec, const LaunchCfg &cfg, const HopArgs &a, int nparity, int epi) {
    if (cfg.nt >= 0) return cfg.nt != 0;
    // links read by one launch (8 slabs) + input, output and epilogue fields
    const double pts = (double)padded(a.npts) * nparity;
    const double ws = 8.0 * (double)a.slab_bytes + pts * spinor_point_bytes(prec) * ((epi & EPI_XPAY) ? 3 : 2);
    return ws > 200e6;
}

unsigned occupancy_lds(int occ, int block, unsigned static_lds) {
    if (occ <= 0) return 0;
    const int waves = block / 64;
    const int per_cu = std::max(1, 4 * occ / waves);  // blocks per CU
    const unsigned total = 160u * 1024u / per_cu;
    // the static LDS of the kernel (block sums) counts against the same budget
    const unsigned dyn = total > static_lds + 256 ? (total - static_lds) & ~255u : 256u;
    return dyn;
}

int effective_tps(int prec, const LaunchCfg &cfg) {
    (void)prec;
    return cfg.tps == 2 ? 2 : 1;
}

template <int SP, int GP, int RECON, int TPS>
static hipError_t launch_batch_tt(bool dag, bool nt, int epi, const BatchArgs &B, dim3 grid, dim3 blk, hipStream_t s) {
#define WL_BATCH_CASE(D, E, N) hipLaunchKernelGGL((hop_batch_kernel<SP, GP, RECON, D, E, N, TPS>), grid, blk, 0, s, B)
    // epilogue bits 0-2, then dagger, then non-temporal stores
    constexpr int DG = 8, NS = 16, CGR = EPI_XPAY | EPI_NORM | EPI_CGR;
    const int key = (dag ? DG : 0) | (nt ? NS : 0) | epi;
    switch (key) {
    case 0: WL_BATCH_CASE(false, 0, false); break;
    case EPI_XPAY: WL_BATCH_CASE(false, EPI_XPAY, false); break;
    case EPI_XPAY | EPI_NORM: WL_BATCH_CASE(false, EPI_XPAY | EPI_NORM, false); break;
    case DG: WL_BATCH_CASE(true, 0, false); break;
    case DG | EPI_XPAY: WL_BATCH_CASE(true, EPI_XPAY, false); break;
    case DG | EPI_XPAY | EPI_NORM: WL_BATCH_CASE(true, EPI_XPAY | EPI_NORM, false); break;
    case DG | CGR: WL_BATCH_CASE(true, CGR, false); break;
    case NS: WL_BATCH_CASE(false, 0, true); break;
    case NS | EPI_XPAY: WL_BATCH_CASE(false, EPI_XPAY, true); break;
    case NS | EPI_XPAY | EPI_NORM: WL_BATCH_CASE(false, EPI_XPAY | EPI_NORM, true); break;
    case NS | DG: WL_BATCH_CASE(true, 0, true); break;
    case NS | DG | EPI_XPAY: WL_BATCH_CASE(true, EPI_XPAY, true); break;
    case NS | DG | EPI_XPAY | EPI_NORM: WL_BATCH_CASE(true, EPI_XPAY | EPI_NORM, true); break;
    case NS | DG | CGR: WL_BATCH_CASE(true, CGR, true); break;
    default: return hipErrorInvalidValue;
    }
#undef WL_BATCH_CASE
    return hipGetLastError();
}

template <int SP, int GP, int RECON>
static hipError_t launch_batch_t(int tps, bool dag, bool nt, int epi, const BatchArgs &B, dim3 grid, dim3 blk,
                                 hipStream_t s) {
    if constexpr (SP == WL_F64 || SP == WL_F32) {
        if (tps == 2) return launch_batch_tt<SP, GP, RECON, 2>(dag, nt, epi, B, grid, blk, s);
    }
    return launch_batch_tt<SP, GP, RECON, 1>(dag, nt, epi, B, grid, blk, s);
}

hipError_t launch_hop_batch(int prec, int recon, bool dagger, int epi, bool nt, int tps, BatchArgs &B, int nwg,
                            int block, hipStream_t stream) {
    if (B.nsys < 1 || B.nsys > BATCH_MAX || block <= 0 || block > 256 || block % 64 || nwg < 8 || nwg % 8 ||
        B.ntiles >= (1L << 30))
        return hipErrorInvalidValue;
    for (int k = 0; k < B.nsys; ++k) {
        HopArgs &a = B.sys[k];
        if (a.npts > (1L << 30)) return hipErrorInvalidValue;  // 32-bit point indices
        a.swizzle = 0;
        a.tchunk = 0;
        a.chunk_sites = 0;
    }
    dim3 grid((unsigned)nwg), blk(block);
    if (prec == WL_F64)
        return recon == 12 ? launch_batch_t<WL_F64, WL_F64, 12>(tps, dagger, nt, epi, B, grid, blk, stream)
                           : launch_batch_t<WL_F64, WL_F64, 18>(tps, dagger, nt, epi, B, grid, blk, stream);
    if (prec == WL_F32)
        return recon == 12 ? launch_batch_t<WL_F32, WL_F32, 12>(tps, dagger, nt, epi, B, grid, blk, stream)
                           : launch_batch_t<WL_F32, WL_F32, 18>(tps, dagger, nt, epi, B, grid, blk, stream);
    if (prec == WL_F16N && recon == 12)
        return launch_batch_t<WL_F16N, WL_F16N, 12>(1, dagger, nt, epi, B, grid, blk, stream);
    if (prec == WL_BF16N && recon == 12)
        return launch_batch_t<WL_BF16N, WL_BF16N, 12>(1, dagger, nt, epi, B, grid, blk, stream);
    if (prec == WL_I16N && recon == 12)
        return launch_batch_t<WL_I16N, WL_I16N, 12>(1, dagger, nt, epi, B, grid, blk, stream);
    return hipErrorInvalidValue;
}

// a.tchunk / a.chunk_sites for a LaunchCfg tchunk value (AUTO resolved from the lattice)
void set_processing_order(HopArgs &a, int tchunk) {
    int tch = tchunk;
    const int ly = a.g.L[1], lz = a.g.L[2], lt = a.g.L[3];
    if (tch == WL_TCHUNK_YZ) {
        if (ly % 2 == 0 && lz % 4 == 0) {
            a.tchunk = WL_TCHUNK_YZ;
            a.yz_by = ly / 2;
            a.yz_bz = lz / 4;
            a.chunk_sites = 0;
            a.f_row = make_fastdiv(a.yz_by * a.g.lxh);
            a.f_slab = make_fastdiv(a.yz_bz * a.yz_by * a.g.lxh);
            a.f_blk = make_fastdiv(lt * a.yz_bz * a.yz_by * a.g.lxh);
            return;
        }
        tch = WL_TCHUNK_AUTO;
    }
    if (tch == WL_TCHUNK_AUTO) tch = lz % 8 == 0 && lz >= 16 ? -(lz / 8) : 0;
    if (tch > 0 && tch < a.g.L[3]) {
        a.tchunk = tch;
        a.chunk_sites = a.tchunk * a.g.L[2] * a.g.sz;
    } else if (tch < 0 && -tch < a.g.L[2]) {
        a.tchunk = tch;
        a.chunk_sites = -a.tchunk * a.g.L[3] * a.g.sz;
        a.f_chunk = make_fastdiv(a.chunk_sites);
        a.f_kplane = make_fastdiv(-a.tchunk * a.g.sz);
    } else {
        a.tchunk = 0;
        a.chunk_sites = 0;
    }
}

static hipError_t launch_hop_prec(int prec, int recon, bool dagger, bool nt, int epi_k, int tps, HopArgs &a,
                                  dim3 grid, dim3 blk, hipStream_t stream) {
    if (prec == WL_F64)
        return recon == 12 ? launch_dag<WL_F64, WL_F64, 12>(dagger, nt, epi_k, tps, a, grid, blk, stream)
                           : launch_dag<WL_F64, WL_F64, 18>(dagger, nt, epi_k, tps, a, grid, blk, stream);
    if (prec == WL_F32)
        return recon == 12 ? launch_dag<WL_F32, WL_F32, 12>(dagger, nt, epi_k, tps, a, grid, blk, stream)
                           : launch_dag<WL_F32, WL_F32, 18>(dagger, nt, epi_k, tps, a, grid, blk, stream);
    if (prec == WL_F16N && recon == 12)
        return launch_dag<WL_F16N, WL_F16N, 12>(dagger, nt, epi_k, tps, a, grid, blk, stream);
    if (prec == WL_BF16N && recon == 12)
        return launch_dag<WL_BF16N, WL_BF16N, 12>(dagger, nt, epi_k, tps, a, grid, blk, stream);
    if (prec == WL_I16N && recon == 12)
        return launch_dag<WL_I16N, WL_I16N, 12>(dagger, nt, epi_k, tps, a, grid, blk, stream);
    return hipErrorInvalidValue;
}

hipError_t launch_hop(int prec, int recon, bool dagger, int epi, HopArgs &a, int nparity,
                      const LaunchCfg &cfg, hipStream_t stream, hipEvent_t ev0, hipEvent_t ev1) {
    const int block = cfg.block;
    if (block <= 0 || block > 256 || block % 64) return hipErrorInvalidValue;
    if (a.npts > (1L << 30)) return hipErrorInvalidValue;  // the kernels index points with 32-bit integers
    const int tps = effective_tps(prec, cfg);
    a.swizzle = cfg.swizzle;
    set_processing_order(a, cfg.tchunk);
    const int rpt = effective_rpt(cfg, a.nrhs, tps);
    if (rpt > 1 && (a.nrhs > 256 || block < 64 || (epi & EPI_CGR))) return hipErrorInvalidValue;
    a.sweep = effective_sweep(cfg, a.nrhs, tps, a.g.L[3], prec);
    dim3 grid((unsigned)hop_launch_blocks(tps, cfg, a.npts, a.nrhs, a.g.L[3], a.g.st, prec), (unsigned)nparity);
    dim3 blk(block);
    const bool nt = use_nontemporal(prec, cfg, a, nparity, epi);
    // Outputs up to 80 MB are written through the caches even when the links are
    // read non-temporally: the next kernel of a solve reads them at once, and they fit
    // in the 256 MB Infinity Cache next to its other fields (FP64 e/o CG at 24^3x48,
    // 64 MB outputs: 2 % faster); larger ones (32^3x64 FP64, 201 MB; multi-rhs fields)
    // stay non-temporal (cached there: 7 % slower).  One point per thread only.
    int epi_k = epi;
    if (nt && !(epi & EPI_CGR) && (double)padded(a.npts) * nparity * spinor_point_bytes(prec) <= 80e6)
        epi_k |= EPI_CACHED_OUT;
    // the block sums of the norm epilogue use up to 4 KB of static LDS (8 KB with rpt 4)
    a.shm = occupancy_lds(cfg.occ, block, 8192);
    if (rpt > 1) {
        hipError_t e = ev0 ? hipEventRecord(ev0, stream) : hipSuccess;
        if (e == hipSuccess) {
            if (rpt == 2) e = launch_hop_r2(prec, recon, dagger, nt, epi, a, grid, blk, stream);
            else if (rpt == 3) e = launch_hop_r3(prec, recon, dagger, nt, epi, a, grid, blk, stream);
            else e = launch_hop_r4(prec, recon, dagger, nt, epi, a, grid, blk, stream);
        }
        if (e == hipSuccess && ev1) e = hipEventRecord(ev1, stream);
        return e;
    }
    t_ev[0] = ev0;
    t_ev[1] = ev1;
    const hipError_t e = launch_hop_prec(prec, recon, dagger, nt, epi_k, tps, a, grid, blk, stream);
    t_ev[0] = t_ev[1] = nullptr;
    return e;
}

}  // namespace wl
