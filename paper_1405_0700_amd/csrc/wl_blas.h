// BLAS-1 and solver-scalar kernels on internal spinor fields.
#pragma once

#include "wl_common.h"

namespace wl {

// Device-resident scalars of one right-hand side of a CG solve.
struct CGScalars {
    double rho;      // ||r||^2 of the current iterate
    double pap;      // <p, A p>
    double alpha;
    double beta;
    double target;   // tol^2 ||b||^2
    double rho_max;  // largest ||r||^2 since the last reliable update (mixed precision)
    int iter;        // iterations done in this solve
    int active;      // 1 while iterating
    int status;      // WL_OK / WL_NOT_CONVERGED / WL_BREAKDOWN
    int maxiter;
    int leaving;     // stopped at the alpha step; leaves the active count at the beta step
    double rho_iter; // ||r||^2 of the iterated residual just before an FP64 refresh
};

struct VecArgs {
    void *v[4][2];     // up to 4 fields, each given per half (half 0 / half 1)
    long n;            // points per half
    int nrhs;
    double a, b;       // scalars (see each kernel)
    double *partials;  // per-block partial sums, rhs r at partials[r * part_stride + block]
    long part_stride;
    CGScalars *sc;     // per-rhs solver scalars (kernels that use them)
    const int *flag;   // if non-null and *flag == 0 (no system still iterating) the launch does nothing
};

// all launchers: nhalves = 1 (EVEN/ODD field) or 2 (FULL field)
hipError_t blas_axpby(int prec, VecArgs &a, int nhalves, bool norm, hipStream_t s);      // v1 = a v0 + b v1 [, ||v1||^2]
hipError_t blas_dot(int prec, VecArgs &a, int nhalves, hipStream_t s);                   // <v0, v1>: re at rhs r, im at rhs nrhs + r
hipError_t blas_norm2(int prec, VecArgs &a, int nhalves, hipStream_t s);                 // ||v0||^2
hipError_t blas_zero(int prec, VecArgs &a, int nhalves, hipStream_t s);                  // v0 = 0
// x += alpha p ; r -= alpha s ; ||r||^2 partials (alpha = sc[rhs].alpha):
// v0 = x (FP64 or low precision, xprec), v1 = p, v2 = r, v3 = s
hipError_t cg_update_xr(int prec, int xprec, VecArgs &a, int nhalves, hipStream_t s);
// p = r + beta p (beta = sc[rhs].beta): v0 = r, v1 = p
hipError_t cg_update_p(int prec, VecArgs &a, int nhalves, hipStream_t s);
// after a hopping launch with EPI_CGR updated r: x += alpha p (where alpha != 0), then
// p = r + beta p (active systems): v0 = x (FP64 solution, or an FP32 accumulator:
// xprec), v1 = p, v2 = r.  Launch it without a flag; cg_alpha zeroes alpha in
// iterations that take no step.
hipError_t cg_update_xp(int prec, int xprec, VecArgs &a, int nhalves, hipStream_t s);
// v1 (prec dprec) = v0 (prec sprec), or v1 += v0 if accumulate
hipError_t blas_convert(int dprec, int sprec, bool accumulate, VecArgs &a, int nhalves, hipStream_t s);
// v1 += (a + i b) v0
hipError_t blas_caxpy(int prec, VecArgs &a, int nhalves, hipStream_t s);
// v1 = a (1 + i b gamma_5) v0
hipError_t blas_twist(int prec, VecArgs &a, int nhalves, hipStream_t s);

// Linear combinations of FP64 fields viewed as arrays of n complex numbers:
// out[o] (+)= sum_j coef[j * nout + o] in[j], each input read once.
constexpr int LC_MAX_IN = 64, LC_MAX_OUT = 32;
struct LinCombArgs {
    const double2 *in[LC_MAX_IN];
    double2 *out[LC_MAX_OUT];
    const double2 *coef;  // device, nin * nout complex
    int nin, nout;
    int accumulate;       // add to out instead of overwriting it
    long n;
};
hipError_t blas_lincomb(const LinCombArgs &a, hipStream_t s);
// Block of inner products C[j][o] = <in[j], w[o]> (j < nin <= 64, o < nw <= 16) of FP64
// fields of n complex numbers, as a tall-skinny product In^+ W on the FP64 matrix
// cores: each wave forms the 64 x 16 product of 16-element slices (four 16 x 16 x 4
// MFMAs per slice and input tile for the complex product), the four waves of a block
// are summed in LDS, and block b leaves re/im of (j, o) at
// partials[(2 (j nw + o) + {0,1}) stride + b] for b < blockdot_blocks(n) <= stride.
constexpr int BD_MAX_IN = 64, BD_MAX_W = 16;
struct BlockDotArgs {
    const double2 *in[BD_MAX_IN];
    const double2 *w[BD_MAX_W];
    int nin, nw;
    long n;
    double *partials;
    long stride;
};
long blockdot_blocks(long n);
hipError_t blas_blockdot(const BlockDotArgs &a, hipStream_t s);
// v1 = v0 / sqrt(sc[0].rho) for one FP64 right-hand side (the normalised residual of a
// CG run; does nothing once *flag == 0)
hipError_t blas_scale_by_rho(VecArgs &a, int nhalves, hipStream_t s);
// Appends (alpha, beta) of sc[0] to hist (ring of `cap` pairs, slot (iter - 1) % cap)
// when sc[0].iter has advanced past *recorded: run after every CG iteration, it keeps
// each iteration's step lengths, the last one's included.
hipError_t cg_record(const CGScalars *sc, double *hist, int cap, int *recorded, hipStream_t s);
// out[v] = sum_b partials[v * stride + b] (b < nblk) for v < nvals, one block per value
hipError_t reduce_rows(const double *partials, long stride, long nblk, int nvals, double *out, hipStream_t s);
// r = b - v  (v2 = r output, v0 = b, v1 = v), ||r||^2 partials: used for true residuals
hipError_t blas_residual(int prec, VecArgs &a, int nhalves, hipStream_t s);

inline int blas_block() { return 256; }
inline long blas_blocks(long n) { return (n + blas_block() - 1) / blas_block(); }

// single-block reductions of `nblk` partials per rhs
//   out[r] = sum_b partials[r * stride + b]   (r < nvals)
hipError_t reduce_partials(const double *partials, long stride, long nblk, int nvals, double *out,
                           hipStream_t s);
// CG scalar steps (one launch each, all rhs):
//   alpha: pap = sum; breakdown check; alpha = rho / pap
//   beta : rho' = sum; convergence / maxiter checks; beta = rho' / rho
// `done` / `flag` point at the number of systems still iterating (one block per
// system; a system that stops decrements it)
hipError_t cg_alpha(CGScalars *sc, int nrhs, const double *partials, long stride, long nblk,
                    const int *flag, hipStream_t s);
//   mode 1: the residual was just refreshed in FP64 (restart the rho_max record;
//           the search direction is restarted too if the refreshed ||r|| is more
//           than twice the iterated one, rho_iter, recorded by cg_stash_rho);
//   mode 2: always restart the search direction (beta = 0)
hipError_t cg_beta(CGScalars *sc, int nrhs, const double *partials, long stride, long nblk, int *done,
                   int mode, hipStream_t s);
// rho_iter = sum(partials) for every active rhs (before an FP64 refresh overwrites them)
hipError_t cg_stash_rho(CGScalars *sc, int nrhs, const double *partials, long stride, long nblk, const int *flag,
                        hipStream_t s);
// initialise: rho = sum(partials) (||r0||^2), target = tol^2 * bnorm2[r]; active if rho > target
hipError_t cg_init(CGScalars *sc, int nrhs, const double *partials, long stride, long nblk,
                   const double *bnorm2, double tol, int maxiter, int *done, hipStream_t s);

// ------------------------------------------------------------------ inner CG on (D M)^+ (D M) y = (D M)^+ rho0
// FP32 fields of nrhs right-hand sides; per-rhs scalars on the device:
//   gam = ||s||^2 with s = (D M)^+ rho, alpha = gam / ||D M p||^2, beta = gam' / gam,
//   rho2 = ||rho||^2 of the system residual rho = rho0 - D M y, stop2 its stopping level.
struct PcgScalars {
    double gam, alpha, beta, rho2, stop2;
    int active;     // 1 while this rhs iterates
    int iters;      // inner iterations taken by this rhs in the current cycle
    int breakdown;  // a non-positive or non-finite step length or norm stopped it
    int pad;
};
struct PcgVec {
    void *y[2], *p[2], *rho[2], *q[2];  // per half of a FULL field
    long n;                             // points per half
    int nrhs;
    PcgScalars *sc;
    double *partials;
    long part_stride;
};
// start of a cycle: gam = sum(partials) (||s||^2), rho2 = rho2_start[r], stop2 = stop2[r]; active where
// live[r] and rho2 > stop2 and gam > 0; *count = number of active rhs
hipError_t pcg_start(PcgScalars *sc, int nrhs, const double *partials, long stride, long nblk,
                     const double *rho2_start, const double *stop2, const int *live, int *count, hipStream_t s);
// alpha = gam / sum(partials) (||D M p||^2) for active rhs (0 else; breakdown stops the rhs)
hipError_t pcg_alpha(PcgScalars *sc, int nrhs, const double *partials, long stride, long nblk, int *count,
                     hipStream_t s);
// y += alpha p, rho -= alpha q, partials of ||rho||^2 (rhs with alpha = 0 unchanged)
hipError_t pcg_update_yr(const PcgVec &v, hipStream_t s);
// rho2 = sum(partials); an active rhs stops once rho2 <= stop2 (or rho2 is not finite); iters += 1
hipError_t pcg_check(PcgScalars *sc, int nrhs, const double *partials, long stride, long nblk, int *count,
                     hipStream_t s);
// beta = sum(partials) / gam (the new ||s||^2), gam = that, for active rhs
hipError_t pcg_beta(PcgScalars *sc, int nrhs, const double *partials, long stride, long nblk, int *count,
                    hipStream_t s);
// p = s + beta p for active rhs (v.p = p, v.q = s)
hipError_t pcg_update_p(const PcgVec &v, hipStream_t s);
// zero the points of the right-hand sides r with mask[r] != 0 in a FULL field of nrhs (storage prec)
hipError_t blas_zero_masked(int prec, void *f, size_t half, long n, int nrhs, const int *mask, hipStream_t s);

}  // namespace wl
