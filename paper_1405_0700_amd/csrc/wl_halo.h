// The hopping term of one output parity computed the way one rank of a lattice
// decomposed in t computes it while its faces are in transit (the paper's scheme
// for overlapping communication with computation): the source field's two
// t-faces are projected to half spinors (the backward one also multiplied by
// U_t^+ on the sending side) and packed; the bulk kernel computes every output
// site from local data, leaving the partial sums of the two boundary slices in
// the output; after the faces have arrived the boundary kernel adds the hops
// that cross them and scales.  Each site's hops are added in the order of the
// fused kernel.
//
// Face buffers: 6 complex numbers of the storage type per face site,
// component-major (component k of face site f at k * fs + f, fs = sites of one
// parity in a t-slice).
#pragma once

#include "wl_dslash.h"

namespace wl {

// storage precision WL_F64 or WL_F32 (the partial sums are kept in the output
// field exactly), one right-hand side, no epilogue (out = b H in)
hipError_t launch_face_pack(int prec, int recon, bool dag, const HopArgs &a, int par, void *send_fwd, void *send_bwd,
                            hipStream_t s);
// nt: non-temporal link loads and output stores; a.swizzle: XCD-aware block order
hipError_t launch_hop_bulk(int prec, int recon, bool dag, bool nt, const HopArgs &a, int par, hipStream_t s);
hipError_t launch_hop_boundary(int prec, int recon, bool dag, const HopArgs &a, int par, const void *recv_fwd,
                               const void *recv_bwd, hipStream_t s);

}  // namespace wl
