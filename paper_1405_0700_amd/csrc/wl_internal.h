// Internal declarations shared by the translation units of the C ABI (context,
// operators, CG, batch / autotuner, EigCG, learned preconditioner): the context
// structure, the error helpers and the host-side helpers each layer uses.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <array>
#include <vector>

#include "wilson.h"
#include "wl_blas.h"
#include "wl_dslash.h"
#include "wl_ptc.h"
#include "wl_access.h"
#include "wl_halo.h"

using namespace wl;

// ------------------------------------------------------------------ errors
namespace wli {
extern thread_local std::string g_err;  // message of the calling thread's last error
wl_status fail(wl_status st, const char *fmt, ...);
}  // namespace wli
using namespace wli;

#define HIP_TRY(call)                                                                            \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess) return fail(WL_ERR_HIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

// ------------------------------------------------------------------ context
enum Slot {
    S_TMP_OP = 0,  // odd temporary of wl_dirac_apply
    S_R, S_P, S_Q, S_S, S_TMP,           // solver fields in the inner precision
    S_RHI, S_THI, S_TMPHI,               // FP64 fields for true residuals
    S_XLO,                               // FP32 accumulator of x steps between refreshes (mixed precision)
    S_PARTIALS, S_SCAL, S_BNORM, S_FLAG,
    S_PTC_H, S_PTC_GH, S_PTC_O, S_PTC_GO, S_PTC_PART, S_PTC_E2,       // PTC workspace
    S_GCR_R, S_GCR_X, S_GCR_Z, S_GCR_W, S_GCR_TMP, S_GCR_RHS,          // FGCR workspace
    S_PCG,                                                             // preconditioned CGNR workspace
    S_FACE,                                                            // t-face send / receive buffers
    S_PCG_SC,                                                          // preconditioned CGNR device scalars
    S_PTC_PATHS,                                                       // PTC two-pass layer: 9 path fields
    S_NSLOTS
};

struct wl_ctx {
    int dims[4];
    double phases[8];
    long V, Vh;
    int device;
    Geom g;
    void *gauge[5][2] = {};  // [prec][recon == 12]
    size_t slab[5][2] = {};
    void *buf[S_NSLOTS] = {};
    size_t buf_bytes[S_NSLOTS] = {};
    void *host_pinned = nullptr;
    size_t host_pinned_bytes = 0;
    LaunchCfg cfg[5];  // hopping-kernel launch configuration per storage precision
    // kernel timing
    bool timing = false;
    int timing_stride = 1;  // record every timing_stride-th hopping launch
    unsigned long timing_seq = 0;
    struct TimedLaunch {
        int key;
        hipEvent_t ev[2];
        int iter;   // CG iteration the launch belongs to (-1: none)
        int cycle;  // CG cycle serial number
    };
    int timing_iter = -1;
    int timing_cycle = 0;
    std::vector<TimedLaunch> timed;
    std::vector<hipEvent_t> event_pool;
    size_t pool_used = 0;
    bool capturing = false;  // no timing events inside a stream capture
    // hipGraph replay of one CG iteration (solver param use_graph)
    hipStream_t own_stream = nullptr;  // capture needs a stream other than the null stream
    hipEvent_t handoff[2] = {nullptr, nullptr};
    hipGraph_t cg_graph = nullptr;
    hipGraphExec_t cg_exec = nullptr;
    std::vector<uintptr_t> cg_graph_key;
    // bulk / boundary split: the stream the face exchange runs on, and its events
    hipStream_t comm_stream = nullptr;
    hipEvent_t halo_ev[2] = {nullptr, nullptr};
};

static inline int timing_key(int prec, int recon, int dagger, int epi) {
    return ((prec * 2 + (recon == 12 ? 1 : 0)) * 2 + (dagger ? 1 : 0)) * 8 + epi;
}

static inline bool prec_ok(int p) { return p >= WL_F64 && p <= WL_I16N; }
static inline bool recon_ok(int prec, int r) {
    if (r != 12 && r != 18) return false;
    if (prec >= WL_F16N && r != 12) return false;
    return true;
}

static inline size_t half_bytes(const wl_ctx *c, int prec, int nrhs) {
    return spinor_point_bytes(prec) * (size_t)padded(c->Vh * (long)nrhs);
}

// ------------------------------------------------------------------ validation helpers
static inline wl_status check_field_args(const wl_ctx *c, int subset, int prec, int nrhs) {
    if (!c) return fail(WL_ERR_ARG, "null context");
    if (subset < WL_EVEN || subset > WL_FULL) return fail(WL_ERR_ARG, "bad subset %d", subset);
    if (!prec_ok(prec)) return fail(WL_ERR_ARG, "bad precision %d", prec);
    if (nrhs < 1 || nrhs > 64) return fail(WL_ERR_ARG, "nrhs %d outside [1, 64]", nrhs);
    return WL_OK;
}
static inline bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }
static inline bool overlap(const void *a, size_t na, const void *b, size_t nb) {
    const char *x = (const char *)a, *y = (const char *)b;
    return x < y + nb && y < x + na;
}


struct wl_ctx;
namespace wli {
// ------------------------------------------------------------------ CG state (CG, batch, EigCG)
struct CGRun {
    wl_ctx *c;
    int op, nrhs, prec, recon, nh;
    double kappa;
    hipStream_t s;
    size_t hb_lo, hb_hi;
    void *x, *r, *p, *q, *sv, *tmp;  // inner precision (x is FP64)
    // mixed precision: the fused iterations add alpha p to this FP32 field, which
    // true_residual folds into x (the only reader of x) before it uses x
    void *xlo;
    size_t hb_xlo;
    const void *b;
    void *rhi, *thi, *tmphi;
    double *partials;
    long stride;
    CGScalars *sc;
    double *bnorm2;
    int *done;
    long nblk_blas;
    int ru_restart;
    double mu;  // twisted mass (0: Wilson)
};

// ------------------------------------------------------------------ shared host helpers
wl_status ensure_buf(wl_ctx *c, int slot, size_t bytes);
wl_status ensure_pinned(wl_ctx *c, size_t bytes);
wl_status get_links(wl_ctx *c, int prec, int recon, const void **ptr, size_t *slab);
VecArgs vec_args(const wl_ctx *c, int prec, int nrhs);
void set_vec(VecArgs &a, int k, const void *base, size_t hb);
const char *launch_problem(int block, int tps, int nt, int rpt, int occ = 0, int sweep = 0);
wl_status fill_hop_args(wl_ctx *c, int prec, int recon, void *out, const void *in, const void *x,
                               int out_subset, int nrhs, double a, double b, double *partials, long part_stride,
                               const int *flag, HopArgs &h, int *np_out, double tm_x = 0.0, double tm_h = 0.0);
void set_cg_residual(const wl_ctx *c, int prec, int nrhs, int out_subset, void *cg_r, const CGScalars *cg_sc,
                            HopArgs &h);
wl_status hop_core(wl_ctx *c, int prec, int recon, bool dag, int epi, void *out, const void *in,
                          const void *x, int out_subset, int nrhs, double a, double b, double *partials,
                          long part_stride, const int *flag, hipStream_t s, long *nblk_out = nullptr,
                          double tm_x = 0.0, double tm_h = 0.0, void *cg_r = nullptr,
                          const CGScalars *cg_sc = nullptr);
wl_status apply_m(wl_ctx *c, int op, bool dag, double kappa, int prec, int recon, int nrhs, void *out,
                         const void *in, void *tmp, double *partials, long stride, const int *flag, hipStream_t s,
                         long *nblk, double mu = 0.0);
wl_status apply_mdag_update_r(wl_ctx *c, int op, double kappa, int prec, int recon, int nrhs, void *r,
                                     const void *in, void *tmp, double *partials, long stride, const int *flag,
                                     hipStream_t s, long *nblk, double mu, const CGScalars *sc);
long part_stride_for(const wl_ctx *c, int nrhs);
wl_status reduce_to_host(wl_ctx *c, int nvals, long stride, long nblk, double *out, hipStream_t s);
// looks up the current device's address of the allocation-free entry points' static scratch array
wl_status scratch_setup(int device);
wl_status true_residual(CGRun &R);
wl_status load_residual(CGRun &R);
wl_status cg_finish_iteration(CGRun &R, bool reliable);
wl_status cg_iteration(CGRun &R, bool reliable);
std::vector<uintptr_t> graph_key(const CGRun &R);
wl_status cg_setup(wl_ctx *c, void *x, const void *b, int op, double kappa, int nrhs, const wl_solver_params &P,
                          hipStream_t s, CGRun &R);
}  // namespace wli
