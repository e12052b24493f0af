/*
 * wilson.h -- C ABI of the MI355X (gfx950) Wilson-operator library.
 *
 * The library applies the Wilson hopping term of Eq. (1) of the paper
 * (Sec. 2),
 *
 *   (H phi)(x) = sum_{mu=0..3} [ U_mu(x) (1 - gamma_mu) phi(x + mu)
 *                              + U_mu(x - mu)^+ (1 + gamma_mu) phi(x - mu) ],
 *
 * in the half-spinor form of Eq. (2), and solves with it.  Everything runs on
 * one GPU with hand-written HIP kernels.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Lattice: extents dims = {Lx, Ly, Lz, Lt}, each even and >= 2; direction
 *   mu = 0, 1, 2, 3 is x, y, z, t; lexicographic site index
 *   lex = x + Lx (y + Ly (z + Lz t)); parity (x + y + z + t) mod 2; V sites,
 *   Vh = V / 2 per parity.
 * Gamma matrices: chiral basis, gamma_mu = [[0, A_mu], [A_mu^+, 0]] with
 *   A = (-i sigma_1, -i sigma_2, -i sigma_3, -1) for mu = x, y, z, t;
 *   gamma_5 = diag(1, 1, -1, -1).
 * Boundary phases: phases[2 mu], phases[2 mu + 1] = (re, im) of z_mu.  A
 *   forward hop that wraps in direction mu (x_mu = L_mu - 1 -> 0) is multiplied
 *   by z_mu, a backward hop that wraps (x_mu = 0 -> L_mu - 1) by conj(z_mu).
 *   Periodic = (1, 0), antiperiodic = (-1, 0).
 * Canonical fields (what a user hands in and gets back), FP64, complex
 *   interleaved (re, im), array-of-structures:
 *     gauge        [lex][mu 4][row 3][col 3]                 (V * 72 doubles)
 *     spinor FULL  [rhs][lex][spin 4][colour 3]              (nrhs * V * 24 doubles)
 *     spinor EVEN / ODD  [rhs][i][spin 4][colour 3], i = 0 .. Vh-1 the sites of
 *                  that parity in increasing lex order (i = lex >> 1).
 * Internal fields: the layout the kernels use (site-major structure of
 *   arrays, right-hand side innermost).  Their size comes from
 *   wl_spinor_bytes(); their content is only meaningful to this library.  A
 *   FULL internal field is the EVEN half followed by the ODD half.
 *
 * Ownership: the caller allocates every field buffer passed to an entry point
 * (device memory, e.g. torch.empty(..., device="cuda")) and keeps ownership;
 * the library never frees caller memory.  A wl_ctx owns its gauge-field copies
 * and its solver workspace.
 *
 * Streams: every call is enqueued asynchronously on the given HIP stream
 * (0 = the null stream) unless stated otherwise.  Calls on one context are not
 * thread-safe.
 *
 * Errors: every function returns a wl_status; none throws or aborts.  A
 * negative status means nothing was enqueued (argument errors) or a HIP call
 * failed; wl_last_error() then returns a message (thread-local).  Positive
 * statuses come from solvers that ran: the result is filled in and the info
 * struct says how far they got.
 */
#ifndef WILSON_H
#define WILSON_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    WL_OK = 0,
    WL_NOT_CONVERGED = 1,   /* solver hit maxiter; x and info are filled in            */
    WL_BREAKDOWN = 2,       /* NaN/Inf or non-positive <p, A p>; x holds the last iterate */
    WL_ERR_ARG = -1,        /* bad argument (null / aliased / misaligned pointer, enum) */
    WL_ERR_DIMS = -2,       /* odd, zero or too large extents                          */
    WL_ERR_HIP = -3,        /* a HIP runtime call failed                               */
    WL_ERR_NOMEM = -4,      /* device allocation failed                                */
    WL_ERR_UNSUPPORTED = -5 /* valid but unsupported combination                       */
} wl_status;

/* Storage precision of internal spinor and link fields.  Arithmetic is FP64 for
 * WL_F64 and FP32 for all others.  The 16-bit formats store each spinor point
 * scaled by its own FP32 norm s = max |component| (s = 0 stores zeros), as
 * IEEE half (F16N), bfloat16 (BF16N) or 16-bit fixed point q = round(32767 v / s)
 * (I16N); 16-bit links are stored unscaled (|U_ij| <= 1), 12-real only. */
typedef enum { WL_F64 = 0, WL_F32 = 1, WL_F16N = 2, WL_BF16N = 3, WL_I16N = 4 } wl_prec;

typedef enum { WL_EVEN = 0, WL_ODD = 1, WL_FULL = 2 } wl_subset;

/* Operators M of the solver:
 *   WL_OP_D     D = 1 - kappa H on the full lattice
 *   WL_OP_DHAT  D_hat = 1 - kappa^2 H_eo H_oe on the even sites (Schur complement) */
typedef enum { WL_OP_D = 0, WL_OP_DHAT = 1 } wl_op;

typedef struct wl_ctx wl_ctx;
typedef struct wl_ptc wl_ptc; /* learned preconditioner (see below) */
typedef struct wl_batch wl_batch; /* several contexts solved together (see below) */
typedef struct wl_eigcg wl_eigcg; /* deflation space of the incremental EigCG solver (see below) */

/* ---------------------------------------------------------------- context */

/* Create a context on the current HIP device.
 *   dims      : {Lx, Ly, Lz, Lt}, all even, >= 2, V <= 2^28.
 *   phases    : 8 doubles, boundary phases z_mu as (re, im).
 *   gauge_host: canonical FP64 gauge field in HOST memory (V * 72 doubles); it is
 *               uploaded and converted once; the caller's buffer is not kept.
 * The FP64 18-real link copy is built here; other link formats are built on
 * first use (or by wl_ctx_prepare_links).  Synchronous. */
wl_status wl_ctx_create(const int dims[4], const double phases[8],
                        const double *gauge_host, wl_ctx **out);
wl_status wl_ctx_destroy(wl_ctx *ctx);

/* Build the link copy used by kernels of storage precision `prec` with
 * `recon` = 18 (all 9 complex entries) or 12 (two rows; the third is rebuilt
 * as the complex conjugate of their cross product).  Synchronous. */
wl_status wl_ctx_prepare_links(wl_ctx *ctx, wl_prec prec, int recon);

/* Launch configuration of the hopping kernel for one storage precision.
 *   block   threads per block: 64, 128, 192 or 256
 *   swizzle 1: reorder blocks so that each of the 8 XCDs (each with its own L2)
 *           processes one contiguous range of the processing order; 0: hardware order
 *   tps     threads per output point: 1 (one thread does all 8 hops) or 2 (the
 *           forward and backward hops run in the two halves of a wavefront,
 *           each half storing two spin components; with 16-bit storage the
 *           halves first agree on the point's norm, so the stored bytes are
 *           those of the one-thread store)
 *   tchunk  processing order of the output sites: 0 = even/odd index order
 *           (t slowest); k > 0 = the lattice is cut into chunks of k time
 *           slices and each chunk is walked with z slowest, so that the
 *           neighbours in t and z of a site are read close together in time;
 *           k < 0 = chunks of -k z-planes over all t, each walked with t
 *           slowest (with the swizzle and Lz = 8 (-k) each XCD walks its own
 *           z-range, its sites' t-neighbours a few planes apart).  Values that
 *           do not cut the lattice (|k| >= the extent) mean 0.
 *           WL_TCHUNK_AUTO (the default): -(Lz / 8) when Lz is a multiple of 8
 *           and at least 16, else 0 (measured: the FP64 half-dslash 8-10 %
 *           faster at 24^3x48 and 32^3x64, the 12-rhs FP32 one 14 %).
 *           WL_TCHUNK_YZ: the (y, z) plane is cut into 2 x 4 blocks of
 *           Ly/2 x Lz/4 x-lines, one per XCD with the swizzle, each walked
 *           with t slowest: a block's neighbours outside it are fewer than a
 *           z-range's (24^3: 36 against 48 x-lines per 72); used when Ly is
 *           even and Lz a multiple of 4, else as AUTO.  Measured back to back
 *           1-4 % faster than AUTO on the FP64 half-dslash, 2 % slower on the
 *           FP16 one, and no faster inside the solves: an autotuner option
 *   nt      1: non-temporal hints on the link loads and output stores (they
 *           keep the single-use link stream from evicting re-read spinors from
 *           L2, but also bypass the Infinity Cache); 0: off; -1: on when the
 *           launch's links and spinor fields exceed 200 MB
 *   rpt     right-hand sides per thread: 1, 2, 3 or 4.  With rpt > 1 (and
 *           tps = 1) a thread computes rpt consecutive right-hand sides of one
 *           site and applies each link it loads to all of them; a launch whose
 *           nrhs is not a multiple of rpt uses one point per thread.
 *   occ     0: no cap; k in 1..8: about k waves per SIMD at most (the launch
 *           reserves unused LDS per block so that fewer blocks fit on a compute
 *           unit; fewer points in flight keep the re-read neighbour spinors
 *           within the XCD's L2).  Default 4 for the 16-bit formats, 0 else.
 *   sweep   0: off; k > 0: time sweep (with tps = 1 and rpt = 1): a thread owns
 *           one point of a time slice and walks k consecutive slices of its
 *           column, keeping the column's input spinors at t - 1, t and t + 1
 *           in registers, so both time hops and the hop inside the x pair
 *           read no memory; blocks tile a slice's points, consecutive blocks
 *           take neighbouring tiles of the same time range.  For many
 *           right-hand sides, whose neighbour spinors otherwise fall out of
 *           L2 before their second use.  FP64 and FP32 storage only (ignored
 *           for the 16-bit formats).  Results are those of tps = 1 bit for
 *           bit.  Measured slower than the default launch on the 12-rhs FP32
 *           half-dslash (354 against 310 us at 24^3x48): an option, off by
 *           default.
 * Results do not depend on block, swizzle, tchunk, nt, occ or sweep; tps changes the
 * summation order of the 8 hops and rpt the compiler's contraction of
 * multiply-adds (rounding only).  Defaults are chosen per
 * precision by measurement (see wl_ctx_get_launch). */
#define WL_TCHUNK_AUTO (-1048576) /* tchunk: the processing order chosen from the lattice */
#define WL_TCHUNK_YZ (-2097152)   /* tchunk: y-z blocks, one per XCD, each walked with t slowest */
typedef struct {
    int block;
    int swizzle;
    int tps;
    int tchunk;
    int nt;
    int rpt;
    int occ;
    int sweep;
} wl_launch;
wl_status wl_ctx_set_launch(wl_ctx *ctx, wl_prec prec, const wl_launch *cfg);
wl_status wl_ctx_get_launch(const wl_ctx *ctx, wl_prec prec, wl_launch *cfg);

/* Bytes of an internal spinor field of `nrhs` right-hand sides. */
wl_status wl_spinor_bytes(const wl_ctx *ctx, wl_subset subset, wl_prec prec,
                          int nrhs, size_t *bytes);

/* canonical FP64 (device) -> internal (device), and back.  For the 16-bit
 * formats pack computes the per-point norm and rounds to nearest even. */
wl_status wl_pack_spinor(const wl_ctx *ctx, void *dst_internal, const double *src_canonical,
                         wl_subset subset, wl_prec prec, int nrhs, void *stream);
wl_status wl_unpack_spinor(const wl_ctx *ctx, double *dst_canonical, const void *src_internal,
                           wl_subset subset, wl_prec prec, int nrhs, void *stream);

/* internal -> internal with a change of storage precision. */
wl_status wl_convert_spinor(const wl_ctx *ctx, void *dst, wl_prec dst_prec, const void *src,
                            wl_prec src_prec, wl_subset subset, int nrhs, void *stream);

/* ---------------------------------------------------------------- operators */

/* out = H in  (Eq. (1)), evaluated through the half-spinor form of Eq. (2).
 *   out_subset = WL_EVEN : out (even field) = H_eo in (in: odd field)
 *   out_subset = WL_ODD  : out (odd field)  = H_oe in (in: even field)
 *   out_subset = WL_FULL : out (full field) = H in    (in: full field)
 * prec/recon select the storage of spinors and links; out and in must not
 * overlap. */
wl_status wl_dslash_apply(const wl_ctx *ctx, void *out, const void *in, wl_subset out_subset,
                          wl_prec prec, int recon, int nrhs, void *stream);

/* out = H^+ in: Eq. (1) with (1 + gamma_mu) on the forward and (1 - gamma_mu)
 * on the backward neighbour (H^+ = gamma_5 H gamma_5).  Arguments as above. */
wl_status wl_dslash_dagger_apply(const wl_ctx *ctx, void *out, const void *in,
                                 wl_subset out_subset, wl_prec prec, int recon, int nrhs,
                                 void *stream);

/* wl_dslash_apply_split: the same out = H in (H^+ in if dagger != 0) for one
 * output parity (subset WL_EVEN or WL_ODD; in is the opposite parity), one
 * right-hand side, FP64 or FP32 storage (recon 18 or 12), computed the way one
 * rank of a lattice decomposed in t computes it with the paper's scheme for
 * overlapping communication with computation (section of that name): the two
 * t-faces of `in` are projected to half spinors (the backward face multiplied by
 * U_t^+ on the sending side) and packed; they are transferred on a second
 * stream while the bulk kernel computes every site from local data; then a
 * boundary kernel adds the hops through the faces to the two boundary slices.
 * On one device the periodic lattice's faces go to itself, so the transfer is a
 * device copy standing in for the neighbour exchange.  Each site's hops are
 * added in the order of the one-thread-per-point fused kernel, so the result
 * equals wl_dslash_apply's with tps = 1 bit for bit (up to FMA contraction
 * choices of the compiler).  Asynchronous on `stream`; the context keeps the
 * face buffers (24 complex numbers per face site) and the second stream;
 * calls that overlap in time on one context race on those buffers.
 * Errors: WL_ERR_ARG for a FULL subset or bad pointers, WL_ERR_UNSUPPORTED for
 * 16-bit storage. */
wl_status wl_dslash_apply_split(const wl_ctx *ctx, void *out, const void *in, wl_subset subset, wl_prec prec, int recon,
                                int dagger, void *stream);

/* out = M in or M^+ in for op = WL_OP_D (FULL fields) or WL_OP_DHAT (EVEN
 * fields).  Uses a context-owned odd-parity temporary for WL_OP_DHAT. */
wl_status wl_dirac_apply(wl_ctx *ctx, void *out, const void *in, wl_op op, int dagger,
                         double kappa, wl_prec prec, int recon, int nrhs, void *stream);

/* Even/odd helpers for solving D x = b through D_hat:
 *   wl_eo_prepare     : bhat_e = b_e + kappa H_eo b_o
 *   wl_eo_reconstruct : x_o    = b_o + kappa H_oe x_e
 * All fields are half (EVEN or ODD) internal fields of precision prec. */
wl_status wl_eo_prepare(const wl_ctx *ctx, void *bhat_e, const void *b_e, const void *b_o,
                        double kappa, wl_prec prec, int recon, int nrhs, void *stream);
wl_status wl_eo_reconstruct(const wl_ctx *ctx, void *x_o, const void *x_e, const void *b_o,
                            double kappa, wl_prec prec, int recon, int nrhs, void *stream);

/* ---------------------------------------------------------------- twisted mass
 *
 * The twisted-mass Wilson operator (the operator of the paper's twisted-mass
 * solver section; its form in hopping-parameter normalisation):
 *   D_tm = A - kappa H,  A = 1 + i nu gamma_5,  nu = 2 kappa mu,
 * D_tm^+ = A^+ - kappa H^+ (A^+ = 1 - i nu gamma_5).  Even/odd:
 *   D_hat_tm = A - kappa^2 H_eo A^-1 H_oe  on even sites,  A^-1 = (1 - i nu gamma_5) / (1 + nu^2),
 *   bhat_e = b_e + kappa H_eo A^-1 b_o,   x_o = A^-1 (b_o + kappa H_oe x_e).
 * The site-diagonal factors are applied in the hopping kernels' epilogue.
 * Arguments, layouts and errors as for wl_dirac_apply / wl_eo_prepare /
 * wl_eo_reconstruct; mu must be finite; mu = 0 gives the Wilson operator.
 * wl_cg_solve takes mu in its parameters. */
wl_status wl_dirac_tm_apply(wl_ctx *ctx, void *out, const void *in, wl_op op, int dagger, double kappa, double mu,
                            wl_prec prec, int recon, int nrhs, void *stream);
wl_status wl_eo_prepare_tm(const wl_ctx *ctx, void *bhat_e, const void *b_e, const void *b_o, double kappa, double mu,
                           wl_prec prec, int recon, int nrhs, void *stream);
wl_status wl_eo_reconstruct_tm(const wl_ctx *ctx, void *x_o, const void *x_e, const void *b_o, double kappa, double mu,
                               wl_prec prec, int recon, int nrhs, void *stream);

/* ---------------------------------------------------------------- BLAS-1 */

/* y = a x + y on internal fields (real a).  */
wl_status wl_blas_axpy(const wl_ctx *ctx, double a, const void *x, void *y, wl_subset subset,
                       wl_prec prec, int nrhs, void *stream);
/* result[2] (host) = <x, y> = sum conj(x) y, accumulated in FP64 in a fixed
 * order (bitwise reproducible).  Synchronises the stream. */
wl_status wl_blas_dot(const wl_ctx *ctx, const void *x, const void *y, wl_subset subset,
                      wl_prec prec, int nrhs, double result[2], void *stream);
/* *result (host) = ||x||^2, FP64, fixed order.  Synchronises the stream. */
wl_status wl_blas_norm2(const wl_ctx *ctx, const void *x, wl_subset subset, wl_prec prec,
                        int nrhs, double *result, void *stream);

/* Allocation-free variant of wl_blas_dot, for callers that cannot allocate
 * device memory or synchronise: code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc.  It computes exactly what
 * wl_blas_dot returns (the same kernels and summation order, bit for bit) and
 * writes it to DEVICE memory: result_dev[0] = Re <x, y>, result_dev[1] =
 * Im <x, y>, summed over the nrhs right-hand sides (result_dev: 2 doubles,
 * 8-byte aligned, caller-owned).  Asynchronous on `stream`; no allocation, no
 * host synchronisation.
 * Limit: its partial sums live in a static device array of 2^20 doubles
 * (8 MiB, one per device, held until the process ends), which must hold
 * 2 nrhs (blocks + 1) values, blocks = ceil(Vh nrhs / 256) per parity of the
 * subset; larger inputs return WL_ERR_ARG without launching anything.  Every
 * call on one device shares that device's array: calls that overlap on one
 * device (on different streams, or from different threads) race and must be
 * ordered by the caller.  Nothing in the array needs clearing: every call
 * writes each partial sum before reading it.
 * Errors: as wl_blas_dot (WL_ERR_ARG for bad arguments, WL_ERR_HIP for a
 * launch failure). */
wl_status wl_blas_dot_noalloc(const wl_ctx *ctx, const void *x, const void *y, wl_subset subset,
                              wl_prec prec, int nrhs, double *result_dev, void *stream);

/* ---------------------------------------------------------------- solvers */

typedef struct {
    double tol;          /* stop when ||b - A x|| <= tol ||b|| (A = M^+ M)            */
    int maxiter;         /* total iteration cap (all restarts)                        */
    int check_every;     /* iterations enqueued between host-side convergence reads  */
    int max_restarts;    /* true-residual restarts after the iterated residual converged */
    wl_prec prec;        /* storage of the inner iteration (WL_F64 = plain FP64 CG)   */
    int recon;           /* 18 or 12                                                  */
    int reliable_every;  /* mixed precision: FP64 residual refresh every this many iters */
    double reliable_delta; /* mixed precision: also refresh when ||r|| < delta * max ||r|| */
    int use_graph;       /* replay each plain iteration from a captured hipGraph        */
    int ru_restart;      /* mixed precision: restart the search direction (p = r) at
                            every FP64 residual refresh; 1 on, 0 off, -1 on for the
                            16-bit formats (whose iterated residual drifts too far
                            for the old direction to stay useful)                    */
    double mu;           /* twisted mass: M = D_tm or D_hat_tm (0: Wilson)             */
} wl_solver_params;

typedef struct {
    int iters;            /* iterations performed (all restarts)       */
    int restarts;         /* true-residual restarts                    */
    int reliable_updates; /* FP64 residual refreshes (mixed precision) */
    double rel_resid;     /* final iterated relative residual          */
    double true_rel_resid;/* final ||b - A x|| / ||b|| recomputed in FP64 */
    double seconds;       /* wall time of the solve                    */
    int fallback;         /* FGCR: 1 if it handed over to plain FP64 CG */
    int fallback_iters;   /* FGCR: iterations of that CG                */
} wl_solver_info;

/* Fill in defaults: tol 1e-10, maxiter 100000, check_every 25, max_restarts 5,
 * prec WL_F64, recon 18, reliable_every 100, reliable_delta 0.1, no graph,
 * ru_restart -1, mu 0.
 * Mixed precision: the FP64 residual is refreshed every reliable_every
 * iterations and whenever ||r|| has dropped by reliable_delta since the last
 * refresh; the iteration of that drop is predicted from the observed decay of
 * ||r|| (no device-to-host read in between).  Between refreshes the solution's
 * steps are summed in an FP32 workspace field of the context and added to the
 * FP64 x at each refresh and before the solve returns. */
void wl_solver_params_default(wl_solver_params *p);

/* Conjugate gradient on the normal equations M^+ M x = b, M = D or D_hat
 * (the paper's solvers around the hopping term of Eq. (1); D = 1 - kappa H and
 * the even/odd Schur complement D_hat = 1 - kappa^2 H_eo H_oe by readings C-4
 * and C-6).  Stops on the iterated residual ||b - A x|| <= tol ||b||, then
 * recomputes it in FP64 and continues from the true residual if it misses tol
 * (reading C-7).  Mixed precision: FP64 reliable updates (reading R-21).
 *   x : in: initial guess, out: solution (internal FP64 field of the op's subset)
 *   b : right-hand side (internal FP64 field), not modified
 *   nrhs right-hand sides are solved as independent systems sharing every
 *   operator application; each stops on its own residual (reading C-13).
 * Synchronous: returns when done.  info may be NULL (else nrhs entries).
 * Returns WL_OK, WL_NOT_CONVERGED (maxiter reached; x and info filled) or
 * WL_BREAKDOWN (a non-finite value or <p, A p> <= 0), or a negative error. */
wl_status wl_cg_solve(wl_ctx *ctx, void *x, const void *b, wl_op op, double kappa, int nrhs,
                      const wl_solver_params *params, wl_solver_info *info, void *stream);

/* Plain FP64 CG for M x = eta with M = D (FULL fields of nrhs right-hand
 * sides), through the normal equations D^+ D x = D^+ eta, stopped on the
 * residual of the system itself, ||eta - D x|| <= tol ||eta|| for every rhs
 * (reading C-7: the criterion every solver of D x = eta is compared on;
 * recomputed in FP64; the normal-equation tolerance is tightened and the CG
 * continued until it holds).  params as for wl_cg_solve; info: nrhs entries
 * (may be NULL), iters counts all CG iterations.  Synchronous. */
wl_status wl_cgnr_solve(wl_ctx *ctx, void *x, const void *eta, double kappa, int nrhs,
                        const wl_solver_params *params, wl_solver_info *info, void *stream);

/* Flexible GCR with restarts, right-preconditioned by the PTC network
 * (reading C-16: FGCR(m) on D; the network by reading C-14).
 * One cycle keeps up to `restart` search directions: z = M(r), w = D z,
 * w and z modified-Gram-Schmidt orthogonalised against the kept pairs,
 * alpha = <w, r> / <w, w>, x += alpha z, r -= alpha w (FP32 fields and FP32
 * arithmetic for D and M, FP64 dot products).  After each cycle the correction
 * is added to the FP64 solution and the residual recomputed in FP64.  Breakdown,
 * non-finite values, two cycles that reduce ||r|| by less than `stagnation`,
 * or maxiter hand the solve to plain FP64 CG (wl_cgnr_solve) if `fallback`. */
typedef struct {
    double tol;        /* stop when ||b - D x|| <= tol ||b||                       */
    int maxiter;       /* preconditioned iterations before giving up              */
    int restart;       /* search directions kept per cycle, 1..64                 */
    int fallback;      /* finish with plain FP64 CG on failure                    */
    double stagnation; /* a cycle must reduce ||r|| below this factor             */
} wl_fgcr_params;

/* tol 1e-10, maxiter 5000, restart 16, fallback 1, stagnation 0.999 */
void wl_fgcr_params_default(wl_fgcr_params *p);

/* Solve D x = b (FULL FP64 fields; x in: initial guess, out: solution) with
 * net == NULL meaning no preconditioner (M = 1).  Synchronous. */
wl_status wl_fgcr_solve(wl_ctx *ctx, void *x, const void *b, double kappa, const wl_ptc *net,
                        const wl_fgcr_params *params, wl_solver_info *info, void *stream);

/* ---------------------------------------------------------------- learned preconditioner */

/* Parallel-transport convolution (PTC) network, two linear layers without
 * bias, 1 -> C -> 1 channels (C <= 16):
 *   out[a](x) = sum_b sum_p W_p^{ab} (T_p in[b])(x),
 * nine paths p: p = 0 the identity, p = 1 + 2 mu the transport
 * U_mu(x) psi(x + mu), p = 2 + 2 mu the transport U_mu(x - mu)^+ psi(x - mu),
 * with the same boundary phases as the Wilson operator; W_p^{ab} are complex
 * 4x4 spin matrices.  Weights: layer 1 (9, C, 1, 4, 4), layer 2 (9, 1, C, 4, 4)
 * complex, row-major, (re, im) interleaved.  The network keeps FP32 master
 * weights (optimised by Adam) and a BF16 copy that its kernels read; fields
 * are FULL FP32 internal fields, a field of C channels being C consecutive
 * single-rhs FULL FP32 fields (channel-major); arithmetic is FP32. */
/* Create a network from host FP64 weights (copied to the device). Synchronous. */
wl_status wl_ptc_create(int channels, const double *w1, const double *w2, wl_ptc **out);
wl_status wl_ptc_destroy(wl_ptc *net);
/* FP32 master weights / accumulated gradients dL/dW* to host FP64 arrays
 * (either pointer may be NULL).  Synchronous. */
wl_status wl_ptc_get_weights(const wl_ptc *net, double *w1, double *w2);
wl_status wl_ptc_get_grads(const wl_ptc *net, double *g1, double *g2);
/* Adam's first and second moments of the real parameters (Re W, Im W) to host
 * FP64 arrays laid out like the weights (layer 1 then layer 2, each entry a
 * (re-part moment, im-part moment) pair; m1 / v1 hold 2 x 9 x C x 16 values,
 * m2 / v2 the same); any pointer may be NULL.  Synchronous. */
wl_status wl_ptc_get_moments(const wl_ptc *net, double *m1, double *m2, double *v1, double *v2);

/* out = M(in) (adjoint == 0) or M^+(in): the two layers with the BF16
 * weights, applied alike to each of nrhs right-hand sides (FULL FP32 fields of
 * nrhs, points (site, rhs) with rhs fastest; the right-hand sides of a site
 * share its link loads). */
wl_status wl_ptc_apply(wl_ctx *ctx, const wl_ptc *net, void *out, const void *in, int nrhs, int adjoint,
                       void *stream);

/* One layer with explicit FP32 device weights `weights` of shape
 * (9, cout_f, cin_f, 4, 4): adjoint == 0 computes out (cout channels) from in
 * (cin channels) with cout_f = cout, cin_f = cin; adjoint != 0 applies the
 * adjoint map g_in[b] = sum_a sum_p T_p^+ W_p^{ab +} g_out[a] of the layer with
 * cout_f = cin, cin_f = cout.  cout * cin <= 16. */
wl_status wl_ptc_layer(wl_ctx *ctx, void *out, const void *in, const float *weights, int cout, int cin,
                       int adjoint, void *stream);

/* grad (device, complex double, shape (9, cout, cin, 4, 4)) = (or +=, if
 * accumulate) dL/d conj(W) = sum_x sum_colour g_out[a](x) (T_p in[b])(x)^+ for a
 * layer with input `in` (cin channels) and output gradient g_out (cout). */
wl_status wl_ptc_weight_grad(wl_ctx *ctx, double *grad, const void *g_out, const void *in, int cout, int cin,
                             int accumulate, void *stream);

/* Training: for one (residual r, error e) pair on this context's gauge field,
 * add inv_npairs * ||M(r) - e||^2 / ||e||^2 to the network's loss and its
 * gradient to the network's gradient accumulators (forward, loss and backward
 * kernels; nothing leaves the device). */
wl_status wl_ptc_accumulate(wl_ctx *ctx, wl_ptc *net, const void *r, const void *e, double inv_npairs,
                            void *stream);
/* Training with the residual-norm loss: for one residual r (FULL FP32, one
 * channel) add inv_npairs * ||D M(r) - r||^2 / ||r||^2 to the loss and its
 * gradient to the accumulators, D = 1 - kappa H of Eq. (1) applied in FP32.
 * For a pair with r = D e this is ||D (M(r) - e)||^2 / ||D e||^2: the pair's
 * error measured by the residual it leaves, the quantity one step x += M(r) of
 * a right-preconditioned Krylov method reduces.  The backward pass applies D^+
 * to the residual and then the adjoint layers. */
wl_status wl_ptc_accumulate_residual(wl_ctx *ctx, wl_ptc *net, const void *r, double kappa, double inv_npairs,
                                     void *stream);
/* One Adam step (beta 0.9, 0.999, eps 1e-8, learning rate lr) with the
 * accumulated gradients; returns the accumulated loss in *loss (may be NULL)
 * and clears both.  Synchronises the stream. */
wl_status wl_ptc_step(wl_ptc *net, double lr, double *loss, void *stream);

/* ---------------------------------------------------------------- preconditioned CGNR
 *
 * CG on the normal equations of the right-preconditioned system D M y = b,
 * x = M y (readings R-20 and C-16), with M the PTC network of `net` (or M = 1
 * for net == NULL): each iteration applies D M and its adjoint M^+ D^+, so
 * (D M)^+ (D M) is Hermitian positive definite whatever the spectrum of D
 * (restarted GCR on D stalls once D's spectrum surrounds the origin, as it
 * does past the critical kappa).  nrhs right-hand sides share every operator
 * and network application (the links and weights are read once for all);
 * each has its own scalars, kept on the device.  The inner iteration runs in
 * FP32 (fields, D, the network) with FP64 dot products, on the correction of
 * the FP64 residual, until that residual has dropped by inner_tol; then
 * x += M y in FP64 and the residual is recomputed in FP64 (defect
 * correction).  Every rhs stops on ||b - D x|| <= tol ||b|| (reading C-7).
 * Two outer cycles that reduce a rhs's ||b - D x|| by less than the factor
 * `stagnation`, breakdown or maxiter mark it failed; failed rhs hand the
 * solve to plain FP64 CG (wl_cgnr_solve, continuing every rhs from its x) if
 * `fallback`.  A zero right-hand side returns x = 0. */
typedef struct {
    double tol;        /* stop when ||b - D x|| <= tol ||b||                      */
    int maxiter;       /* inner iterations in total                              */
    double inner_tol;  /* residual reduction per outer cycle, in (0, 1)          */
    int fallback;      /* finish with plain FP64 CG on failure                   */
    double stagnation; /* an outer cycle must reduce ||r|| below this factor     */
} wl_pcgnr_params;

/* tol 1e-10, maxiter 20000, inner_tol 1e-5, fallback 1, stagnation 0.5 */
void wl_pcgnr_params_default(wl_pcgnr_params *p);

/* Solve D x = b (FULL FP64 fields of nrhs right-hand sides; x in: initial
 * guess, out: solution).  Synchronous; info: nrhs entries or NULL (iters =
 * inner iterations, restarts = outer cycles, fallback / fallback_iters). */
wl_status wl_pcgnr_solve(wl_ctx *ctx, void *x, const void *b, double kappa, const wl_ptc *net, int nrhs,
                         const wl_pcgnr_params *params, wl_solver_info *info, void *stream);

/* ---------------------------------------------------------------- batches of systems
 *
 * A batch groups 1..8 contexts on one device (lattices of any, also different,
 * sizes, each with its own gauge field).  Their hopping-term launches are
 * merged into ONE persistent launch per operator stage: the blocks of points
 * of all systems form one work list, split into eight contiguous ranges (one
 * per XCD, so that an XCD's L2 sees neighbouring tiles of one lattice), which
 * a fixed grid of resident workgroups of that XCD takes round-robin (every
 * tile costs the same; no device state persists between launches, so a
 * launch can be replayed inside a graph).  The batch owns a non-blocking
 * stream used for graph capture; it does not own the contexts, which must
 * outlive it.  Calls on one batch are not thread-safe. */
wl_status wl_batch_create(wl_ctx *const *ctxs, int nsys, wl_batch **out);
wl_status wl_batch_destroy(wl_batch *batch);
/* Persistent workgroups (a multiple of 8; default 3 per compute unit),
 * threads per tile (64..256, a multiple of 64; default 256), non-temporal
 * hints (1 on, 0 off, -1 by working-set size, the default) and threads per
 * output point (1, the default; 2: forward and backward hops in the two halves
 * of a wavefront, for FP64 / FP32 storage only, measured slower here).
 * workgroups = 0 replaces the persistent launch by one launch per system and
 * stage, each with its context's own launch configuration (block, nt and tps
 * are then unused; the batch timing calls record nothing, the contexts' own
 * timing does): faster when every system fills the GPU by itself. */
wl_status wl_batch_set_launch(wl_batch *batch, int workgroups, int block, int nt, int tps);
wl_status wl_batch_get_launch(const wl_batch *batch, int *workgroups, int *block, int *nt, int *tps);

/* out[k] = M_k in[k] (M_k^+ if dagger) for every system k of the batch, M = D
 * (FULL fields) or D_hat (EVEN fields), kappa[k] per system, all fields in
 * precision prec with nrhs right-hand sides (same for every system).
 * Asynchronous on `stream`. */
wl_status wl_batch_dirac_apply(wl_batch *batch, void *const *out, const void *const *in, wl_op op, int dagger,
                               const double *kappa, wl_prec prec, int recon, int nrhs, void *stream);

/* CG on the normal equations M_k^+ M_k x[k] = b[k] of every system together
 * (readings C-7 and C-13 as for wl_cg_solve, per system and rhs;
 * the independent solves of each system's nrhs right-hand sides run in
 * lockstep: one persistent launch per hopping stage of an iteration, the
 * scalar and vector steps per system).  Parameters as for wl_cg_solve (inner
 * precision, FP64 reliable updates, use_graph: the lockstep iteration is
 * captured in one graph on the batch's own stream and replayed).  A system
 * whose right-hand sides have all converged drops out of the persistent
 * launches.  info: nsys * nrhs entries, system-major.  Synchronous. */
wl_status wl_batch_cg_solve(wl_batch *batch, void *const *x, const void *const *b, wl_op op, const double *kappa,
                            int nrhs, const wl_solver_params *params, wl_solver_info *info, void *stream);

/* Event timing of the batch's persistent launches (as wl_timing_enable /
 * wl_timing_read for a context, all launches of the batch together). */
wl_status wl_batch_timing_enable(wl_batch *batch, int enable);
wl_status wl_batch_timing_read(wl_batch *batch, int *count, double *total_ms);

/* ---------------------------------------------------------------- autotuner
 *
 * Times the hopping-term launch the solvers use (out = x - kappa H in over
 * both parities, on scratch fields the call allocates and frees) for every
 * launch shape of the sweep -- block 64/128/256, one or two threads per point
 * (FP64/FP32 storage) or 2-4 right-hand sides per thread (when nrhs allows),
 * XCD swizzle off/on, processing order by e/o index, by chunks of 4 time
 * slices, by z-ranges (WL_TCHUNK_AUTO) or by y-z blocks (WL_TCHUNK_YZ),
 * non-temporal hints off/on -- with HIP
 * events (average of 5 launches after a warm-up), picks the fastest and makes
 * it the context's launch configuration for `prec`.  Results are cached in
 * the process and, if cache_path is not NULL, appended to that text file
 * (one line per key: GPU architecture, extents, prec, recon, nrhs); a later
 * call with a cached key applies the entry without timing (*from_cache = 1).
 * A file entry that is not a valid launch shape (as wl_ctx_set_launch would
 * reject it) is ignored and the key tuned again; so are unreadable lines.
 * chosen, best_us (microseconds per launch) and from_cache may be NULL.
 * Synchronous. */
wl_status wl_autotune(wl_ctx *ctx, wl_prec prec, int recon, int nrhs, const char *cache_path, wl_launch *chosen,
                      double *best_us, int *from_cache);
/* The same for a batch: one launch per system (workgroups 0, the contexts'
 * current shapes) against the persistent launch with 1..8 workgroups per
 * compute unit (scaled by 256 / block), threads per tile 64/128/256,
 * non-temporal hints and one or two threads per point, all timed on D over
 * every system; the result becomes the batch's launch configuration.  Cache
 * entries that wl_batch_set_launch would reject are ignored. */
wl_status wl_batch_autotune(wl_batch *batch, wl_prec prec, int recon, int nrhs, const char *cache_path,
                            int *workgroups, int *block, int *nt, int *tps, double *best_us, int *from_cache);

/* ---------------------------------------------------------------- incremental EigCG
 *
 * The paper's solver for many right-hand sides of the twisted-mass operator
 * (section on EigCG for twisted-mass fermions; algorithm of Stathopoulos and
 * Orginos): CG on A = M^+ M (M = D or D_hat, optionally twisted, FP64) that
 * also keeps a search space of m normalised residuals (the Lanczos vectors of
 * the CG run) and the real tridiagonal matrix built from CG's alpha and beta;
 * when the space is full it is restarted with the nev lowest Ritz vectors of
 * T_m and of T_{m-1}.  At convergence the nev lowest Ritz vectors are
 * orthonormalised into a growing deflation space U (up to max_vectors), with
 * H = U^+ A U kept on the host.  Every solve starts from the Galerkin guess
 * x0 = U H^-1 U^+ b (init-CG), which removes the error along the computed low
 * modes.  The small dense eigenproblems (m <= 64) and the Cholesky solve with
 * H run on the host; all field operations run on the device: fused kernels
 * form linear combinations of up to 64 fields, and blocks of up to 64 x 16
 * inner products <u_j, w_o> in one pass (on the FP64 matrix cores); they serve
 * the restarts, the init-CG projection, the block classical Gram-Schmidt (two
 * passes) of the new vectors against U, and the new columns of H.
 *
 * wl_eigcg_create: op, kappa and mu fix A; 1 <= nev <= 16, 2 nev + 2 <= m <= 64;
 *   allocates (2 m + 5 + 2 max_vectors) FP64 fields of op's subset.
 * wl_eigcg_solve: solves A x = b (x: output, the input value is ignored)
 *   to ||b - A x|| <= tol ||b|| (FP64 true residual; up to 4 restarts from it),
 *   adding nev vectors to U if collect != 0 and there is room; otherwise (no
 *   vectors to collect) it runs wl_cg_solve's FP64 CG from the init-CG guess.
 *   info: iters (all cycles), restarts, rel_resid, true_rel_resid, seconds.
 *   Synchronous.
 * wl_eigcg_vectors: number of vectors kept and their Rayleigh quotients
 *   u^+ A u (ritz may be NULL, else room for max_vectors doubles).
 * wl_eigcg_eigenvalues: the Ritz values of A on the whole deflation space, the
 *   eigenvalues of H = U^+ A U in ascending order (*n = number of vectors;
 *   vals may be NULL, else room for max_vectors doubles).  Host-side, O(n^3). */
wl_status wl_eigcg_create(wl_ctx *ctx, wl_op op, double kappa, double mu, int nev, int m, int max_vectors,
                          wl_eigcg **out);
wl_status wl_eigcg_destroy(wl_eigcg *e);
wl_status wl_eigcg_solve(wl_eigcg *e, void *x, const void *b, double tol, int maxiter, int collect,
                         wl_solver_info *info, void *stream);
wl_status wl_eigcg_vectors(const wl_eigcg *e, int *nvec, double *ritz);
wl_status wl_eigcg_eigenvalues(const wl_eigcg *e, int *n, double *vals);

/* ---------------------------------------------------------------- link-spinor access kernel
 *
 * The paper's isolated link-spinor multiplication, used there to compare ways
 * of addressing the sites (section on overlapping communication with
 * computation: sequential access, access through an index array, and access
 * through pointer arrays prepared beforehand).  For i < n:
 *     psi(x_i) = U(x_i) phi(x_i),
 * U a 3x3 complex matrix applied to each of the four colour vectors of the
 * spinor phi; FP64 throughout, all arrays in device memory.
 *   mode WL_ACCESS_SEQ   : x_i = i
 *   mode WL_ACCESS_INDEX : x_i = index[i] (int32 device array of n site numbers
 *                          < the arrays' site count; a permutation writes every
 *                          psi once, a repeated site is written more than once)
 *   mode WL_ACCESS_PTR   : ptrs[3 i], ptrs[3 i + 1], ptrs[3 i + 2] (uint64 device
 *                          array) are the device addresses of psi(x_i), U(x_i) and
 *                          phi(x_i); psi, u, phi are not read (may be NULL)
 *   layout 0: site x of U at u + 144 x bytes (row-major 3x3, re/im
 *             interleaved), of phi/psi at + 192 x (spin-major, colour-minor);
 *   layout 1: blocks of 64 sites, component k of site x at
 *             base + ((x / 64) * 64 * nc + k * 64 + x % 64) * 16 bytes (nc = 9
 *             for U, 12 for spinors); the arrays hold whole blocks.  In pointer
 *             mode the address is that of component 0 (+ k * 1024 for component k).
 * Errors: WL_ERR_ARG for n < 0 or > 2^31 - 1, a bad mode or layout, a missing
 * index / address array, null or misaligned field pointers.  Asynchronous on
 * `stream`. */
typedef enum { WL_ACCESS_SEQ = 0, WL_ACCESS_INDEX = 1, WL_ACCESS_PTR = 2 } wl_access_mode;
wl_status wl_su3_apply(void *psi, const void *u, const void *phi, long n, int mode, int layout, const int *index,
                       const unsigned long long *ptrs, void *stream);

/* ---------------------------------------------------------------- kernel timing */

/* While enabled (enable = n >= 1), every n-th launch of the hopping-term kernel
 * made through this context (by the operators and the solvers; n = 1: every
 * launch) is timed by a pair of HIP events on the stream it is launched on.
 * The kernel's own dispatch packet stamps them at the start and the end of its
 * execution (hipExtLaunchKernelGGL), so that a duration is what a kernel trace
 * reports for the launch; the kernels with several right-hand sides per thread
 * have the events recorded before and after them, which adds the dispatch gaps
 * (a few microseconds).  Sampling (n coprime to the launches of one solver
 * iteration) keeps the instrumented run close to an uninstrumented one.
 * enable = 0 disables.  Enabling (or disabling) discards what was recorded.
 * At most 1 << 16 launches are recorded.  Errors: WL_ERR_ARG for enable < 0. */
wl_status wl_timing_enable(wl_ctx *ctx, int enable);

/* Number and summed GPU duration (milliseconds) of the recorded launches of
 * the hopping kernel with the given storage precision, link format, dagger
 * flag and epilogue (0 = plain out = H in; 1 = out = a x + b H in;
 * 3 = the same plus the fused ||out||^2).  Synchronises on the recorded events. */
wl_status wl_timing_read(wl_ctx *ctx, wl_prec prec, int recon, int dagger, int epilogue, int *count,
                         double *total_ms);

/* ---------------------------------------------------------------- misc */

/* Thread-local message of the last failing call ("" if none). */
const char *wl_last_error(void);

/* Library version string. */
const char *wl_version(void);

#ifdef __cplusplus
}
#endif

#endif /* WILSON_H */
