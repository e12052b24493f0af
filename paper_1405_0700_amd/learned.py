"""Training data and training loop of the learned (PTC) preconditioner.

Argument marshalling and bookkeeping only: every field operation below is a
call into the HIP library (plain CG, Dirac operator, BLAS, the PTC forward /
backward / Adam kernels).

Training pairs: for a source eta, plain FP64 CG on the normal equations of
D x = eta is run from x0 = 0; its iterates x_k at the snapshot iterations give
the pairs (r_k, e_k) with r_k = eta - D x_k (the residual the preconditioner
sees) and e_k = x* - x_k (the error it should return), x* the converged
solution.  Two losses over the pairs, both minimised with Adam on the FP32
master weights:
  error norm     L = (1/N) sum ||M(r) - e||^2 / ||e||^2
  residual norm  L = (1/N) sum ||D (M(r) - e)||^2 / ||D e||^2
                   = (1/N) sum ||D M(r) - r||^2 / ||r||^2      (r = D e)
Which iterations the pairs come from decides what the network learns.  Late
iterations leave residuals and errors made of the smooth low modes of D, which
a network of one-hop transports cannot invert; fitted to them, the error norm
amplifies those modes and the residual norm shrinks them, and either way the
conditioning of D M, which is what CG on its normal equations needs, gets
worse (measured: a net trained on iterations 5..160 takes 578 CG iterations
where no net takes 265, 16^3x32 at kappa 0.137).  The source itself (k = 0:
x_0 = 0, so r = eta, a Gaussian field holding every mode, and e = x*) is the
best input: fitted to it, the residual norm approximates D^-1 where a local
operator can and leaves D M close to the identity elsewhere (measured at
32^3x64: 87 iterations against 303 without a net and 470 with the untrained
one; pairs from iterations 0-1 give 90, 0-3 give 100).  The defaults are the
source alone and the residual norm.
"""

from __future__ import annotations

import time

from . import wilson as W

SNAPSHOTS = (0,)


def harvest(lat, sources, kappa, snapshots=SNAPSHOTS, tol=1e-12):
    """-> list of (r, e) FULL FP32 internal fields (torch tensors) for the given sources."""
    pairs = []
    ctx = lat.ctx
    for eta_c in sources:
        eta = lat.pack(eta_c, W.WL_FULL)
        xs = lat.new(W.WL_FULL)
        p = W.wl_solver_params_default()
        p.tol = tol
        W.wl_cgnr_solve(ctx, xs, eta, kappa, p)
        rhs = lat.new(W.WL_FULL)
        W.wl_dirac_apply(ctx, rhs, eta, W.WL_OP_D, True, kappa)
        for k in snapshots:
            q = W.wl_solver_params_default()
            q.tol, q.maxiter, q.max_restarts = 0.0, int(k), 0
            xk = lat.new(W.WL_FULL)
            W.wl_cg_solve(ctx, xk, rhs, W.WL_OP_D, kappa, params=q)
            e = xs.clone()
            W.wl_blas_axpy(ctx, -1.0, xk, e, W.WL_FULL)
            dx = lat.new(W.WL_FULL, zero=False)
            W.wl_dirac_apply(ctx, dx, xk, W.WL_OP_D, False, kappa)
            r = eta.clone()
            W.wl_blas_axpy(ctx, -1.0, dx, r, W.WL_FULL)
            r32 = lat.new(W.WL_FULL, W.WL_F32, zero=False)
            e32 = lat.new(W.WL_FULL, W.WL_F32, zero=False)
            W.wl_convert_spinor(ctx, r32, W.WL_F32, r, W.WL_F64, W.WL_FULL)
            W.wl_convert_spinor(ctx, e32, W.WL_F32, e, W.WL_F64, W.WL_FULL)
            pairs.append((r32, e32))
    return pairs


def train(sets, net, epochs, lr=1e-3, log=None, loss="residual", kappa=None):
    """sets: list of (lattice, pairs).  One Adam step per lattice per epoch (its
    pairs form the batch).  loss: "residual" (needs kappa), "error", or "both"
    (their sum).
    Returns the loss of every step."""
    if loss not in ("residual", "error", "both"):
        raise ValueError("loss must be 'residual', 'error' or 'both'")
    if loss != "error" and kappa is None:
        raise ValueError("the residual-norm loss needs kappa")
    losses = []
    t0 = time.perf_counter()
    for ep in range(epochs):
        for lat, pairs in sets:
            inv = 1.0 / len(pairs)
            for r, e in pairs:
                if loss != "error":
                    W.wl_ptc_accumulate_residual(lat.ctx, net, r, kappa, inv)
                if loss != "residual":
                    W.wl_ptc_accumulate(lat.ctx, net, r, e, inv)
            losses.append(W.wl_ptc_step(net, lr))
        if log is not None and (ep % max(1, epochs // 10) == 0 or ep == epochs - 1):
            log("epoch %d loss %.5f (%.1f s)" % (ep, losses[-1], time.perf_counter() - t0))
    return losses
