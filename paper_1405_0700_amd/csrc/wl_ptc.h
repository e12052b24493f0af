// Kernels of the parallel-transport convolution (PTC) preconditioner.
#pragma once

#include "wl_common.h"

namespace wl {

constexpr int PTC_NPATH = 9;
constexpr int PTC_MAXC = 16;  // most channels of a layer

// One PTC layer on FULL FP32 fields.  A field of C channels is C consecutive
// FULL fields of nrhs right-hand sides each (channel-major: channel b, parity
// par starts at byte (2 b + par) * half; inside, points (site, rhs) with rhs
// fastest, as every multi-rhs field), so the threads of a wave, one per point,
// read and write consecutive points of each channel; the right-hand sides of
// a site share its links.  The network acts on every right-hand side alike.
//   out[a](x) = sum_b sum_p W_p^{ab} (T_p in[b])(x),  or its adjoint
// g_in[b] = sum_a sum_p T_p^+ W_p^{ab +} g_out[a]  (adjoint != 0; then
// `cout`/`cin` are the channel counts of the adjoint map and the weights keep
// the layout of the forward layer).
struct PtcArgs {
    Geom g;
    const char *in;
    char *out;
    size_t half;        // bytes of one parity of one channel
    const void *gauge;  // FP32 18-real links
    size_t slab_bytes;
    const void *w;      // [9][cout_f][cin_f][4][4] complex, FP32 or BF16 (re, im interleaved)
    int cout, cin;      // channels of this launch's output / input
    int adjoint;
    long vh;
    int nrhs;           // right-hand sides per channel (1 for the training kernels)
    char *paths;        // optional workspace of 9 FULL fields of nrhs (2 * 9 * half bytes): with it a
                        // layer with one output channel (cin > 1) runs in two passes, the channel
                        // mixing of every path at the source point first, then the transports
};

hipError_t launch_ptc_layer(const PtcArgs &a, bool bf16_weights, hipStream_t s);

// The whole two-layer network 1 -> C -> 1 (C = 4 or 8) on matrix cores, in two
// passes: at every point y the nine transports of in, the first layer's channel
// mixing and the second layer's mixing of each path (both real matrix products
// on MFMA with BF16 operands, the FP32 activations split exactly into three BF16
// parts, FP32 accumulation), stored as the nine path fields a.paths; then the
// gather k_ptc_gather into a.out.  Forward (M) or adjoint (M^+) by the table.
// `tab` holds the MFMA operand tables of both layers for one direction, built by
// launch_ptc_net_tables; a.w is not used.  a.cout = a.cin = 1, a.nrhs as usual.
bool ptc_net_supported(int channels);
long ptc_net_table_elems(int channels);  // BF16 elements of one direction's table
hipError_t launch_ptc_net_tables(const uint16_t *wb, long n1, int channels, uint16_t *tab_fwd, uint16_t *tab_adj,
                                 hipStream_t s);
hipError_t launch_ptc_net(const PtcArgs &a, int channels, const uint16_t *tab, hipStream_t s);

// Weight gradient dL/d conj(W_p^{ab}) = sum_x sum_colour g[a](x) (T_p in[b])(x)^+
// for all (p, a, b): per-chunk FP32 partials, then an FP64 sum over chunks that
// is stored to (or added to) grad[p][a][b][4][4] (complex double).  Channel-major
// fields as for the layer.
struct PtcGradArgs {
    Geom g;
    const char *gout;     // cout channels
    const char *in;       // cin channels
    size_t half;
    const void *gauge;
    size_t slab_bytes;
    int cout, cin;
    long vh;
    float *partials;      // [combo][chunk][32]
    int nchunks;
};
hipError_t launch_ptc_wgrad(const PtcGradArgs &a, double *grad, int accumulate, hipStream_t s);

// Loss of one pair: d = out - e, g = scale * d with scale = inv_n / ||e||^2,
// loss += scale * ||d||^2 (all on the device).  e2 must hold ||e||^2.
hipError_t launch_ptc_loss(const void *out, const void *e, void *g, long npts_half, const double *e2,
                           double inv_n, double *partials, long stride, double *loss, hipStream_t s);

// Adam on n real parameters (complex weights as (re, im)); grad_c is the
// complex dL/dW* (double), the real-parameter gradient is 2 grad_c.  Writes the
// FP32 master weights and their BF16 copy, then clears grad_c.
hipError_t launch_adam(float *w, uint16_t *wb, double *grad_c, float *m, float *v, long n, double lr, double b1,
                       double b2, double eps, int t, hipStream_t s);

// FP32 -> BF16 copy of n floats
hipError_t launch_to_bf16(const float *w, uint16_t *wb, long n, hipStream_t s);

}  // namespace wl
