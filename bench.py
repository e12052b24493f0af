#!/usr/bin/env python3
"""Benchmark of the hot path: even/odd preconditioned Wilson CG on one MI355X.

Workload (default): 24^3 x 48 lattice, links exp(0.2 i H) (seeded Gaussian
traceless Hermitian H, reunitarised; seed 201), Gaussian source (seed 202),
kappa = 0.135, periodic in space and antiperiodic in time, FP64 storage and
arithmetic, 18-real links.

One step solves D x = eta through the Schur complement D_hat = 1 - kappa^2 H_eo H_oe:
  bhat = b_e + kappa H_eo b_o;  rhs = D_hat^+ bhat;
  CG on D_hat^+ D_hat x_e = rhs to ||rhs - A x_e|| <= 1e-10 ||rhs||;
  x_o = b_o + kappa H_oe x_e.
All of it runs in the library's kernels; inputs are resident in HBM before the
timed region starts.

Reported:
  value      whole-step throughput in GB/s = algorithmic bytes of every kernel
             of the step (table in `step_bytes`) / step time;
  roofline   the dominant kernel (the plain FP64 half-dslash, 1536 B per output
             site) timed live with HIP events on its own stream over the timed
             region: achieved = 1536 * Vh / average launch duration;
  cpu_baseline  the FP64 CPU oracle running a bounded sample of the same CG
             (fixed iterations) on the host cores, in the same unit.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, AMD published
SITE_BYTES = {  # algorithmic bytes per output site of one half-dslash, FP64 storage, 18-real links
    "hop": 8 * 144 + 192 + 192,          # 8 links + input spinor once + output spinor
    "hop_xpay": 8 * 144 + 3 * 192,       # + the epilogue field x
}
WORKLOAD = dict(dims=(24, 24, 24, 48), eps=0.2, gauge_seed=201, src_seed=202, kappa=0.135,
                phases=(1, 1, 1, -1), tol=1e-10)
PROFILE_DIR = os.path.join(ROOT, "profiles")
TRAFFIC_FILE = os.path.join(PROFILE_DIR, "hop_f64_24x24x24x48_traffic.txt")
KERNEL_SOURCES = ["paper_1405_0700_amd/csrc/wl_dslash.hip", "paper_1405_0700_amd/csrc/wl_dslash.h",
                  "paper_1405_0700_amd/csrc/wl_dslash_kernels.h", "paper_1405_0700_amd/csrc/wl_common.h"]


def step_bytes(vh: int, iters: int, restarts: int) -> int:
    """Algorithmic HBM bytes of one step (FP64 storage, 192 B per spinor site):

      eo_prepare (hop + x read)                   1728
      rhs = D_hat^+ bhat (hop, hop+x)             1536 + 1728
      ||rhs||^2                                    192
      per CG cycle (1 + restarts):
        true residual b - A x at start and end:   2 x (2 x 1536 + 2 x 1728 + 576)
        p = r copy                                  384
      per CG iteration:
        q = D_hat p (hop, hop+x, fused norm)      1536 + 1728
        r -= a D_hat^+ q (hop, hop+x with r read+write in place of the output, fused norm)
                                                  1536 + 1728 + 192
        x += a p, p = r + b p (x, p read+write; r read)    960
      eo_reconstruct (hop + x read)               1728
    per even site; the single-block scalar kernels are not counted.
    """
    h, hx = SITE_BYTES["hop"], SITE_BYTES["hop_xpay"]
    true_res = 2 * h + 2 * hx + 576
    per_iter = 2 * h + 2 * hx + 192 + 960
    fixed = hx + (h + hx) + 192 + hx
    per_cycle = 2 * true_res + 384
    return vh * (fixed + (1 + restarts) * per_cycle + iters * per_iter)


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def read_traffic():
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source; else None."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    for line in open(TRAFFIC_FILE):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256") != kernel_hash():
        return None
    try:
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def make_inputs(wl):
    from paper_1405_0700_amd import synth
    u = synth.su3_links(wl["dims"], wl["eps"], wl["gauge_seed"])
    eta = synth.gaussian_spinor(wl["dims"], wl["src_seed"])
    return u, eta


def cpu_baseline(u, eta, wl, sample_iters, one_thread_iters=2, converge=True):
    """The FP64 oracle on the host cores: a bounded sample (fixed CG iterations on the same Schur
    system, all threads), the same sample on one thread (fewer iterations), and plain oracle CG to
    1e-10 on the 8^4 D^+ D system and on this 24^3x48 Schur system; all timed."""
    import numpy as np

    from oracle import oracle as orc
    from paper_1405_0700_amd import synth
    dims, kappa, ph = wl["dims"], wl["kappa"], wl["phases"]
    be, bo = orc.eo_split(eta, dims)
    bhat = orc.eo_prepare(be, bo, u, kappa, ph)
    rhs = orc.schur(bhat, u, kappa, ph, dagger=True)
    apply_a = lambda v: orc.schur(orc.schur(v, u, kappa, ph), u, kappa, ph, dagger=True)
    vh = be.shape[0]

    def sample_bytes(iters):
        # the sample's algorithmic bytes: iterations + its final true-residual check
        return vh * (iters * (2 * SITE_BYTES["hop"] + 2 * SITE_BYTES["hop_xpay"] + 1152 + 576)
                     + 2 * SITE_BYTES["hop"] + 2 * SITE_BYTES["hop_xpay"] + 576)

    threads = orc.max_threads()
    t0 = time.perf_counter()
    orc.cg(apply_a, rhs, fixed_iters=sample_iters)
    dt = time.perf_counter() - t0
    out = {"value": round(sample_bytes(sample_iters) / dt / 1e9, 4), "unit": "GB/s", "cores": threads,
           "kind": "oracle", "model": host_cpu_model(),
           "sample": "%d fixed CG iterations on D_hat^+ D_hat (24^3x48, FP64) plus its final residual check, "
                     "%.1f s on %d threads" % (sample_iters, dt, threads)}
    orc.set_threads(1)
    try:
        t0 = time.perf_counter()
        orc.cg(apply_a, rhs, fixed_iters=one_thread_iters)
        dt1 = time.perf_counter() - t0
    finally:
        orc.set_threads(threads)
    out["one_thread"] = {"value": round(sample_bytes(one_thread_iters) / dt1 / 1e9, 4), "unit": "GB/s",
                         "sample": "%d fixed CG iterations plus the final residual check, %.1f s on 1 thread"
                                   % (one_thread_iters, dt1)}
    if converge:
        conv = {}
        # config 1: 8^4, links exp(0.5 i H) seed 101, source seed 102, kappa 0.12, full D, CG on D^+ D
        d1 = (8, 8, 8, 8)
        u1 = synth.su3_links(d1, 0.5, 101)
        b1 = synth.gaussian_spinor(d1, seed=102)
        t0 = time.perf_counter()
        _, inf1 = orc.cg_normal(lambda v: orc.dirac(v, u1, 0.12, ph), lambda v: orc.dirac(v, u1, 0.12, ph, True),
                                b1, tol=1e-10)
        conv["8^4_full_D"] = {"seconds": round(time.perf_counter() - t0, 3), "iters": inf1["iters"],
                              "true_rel_resid": float("%.4g" % inf1["true_rel_resid"])}
        # config 2: this 24^3x48 Schur system
        t0 = time.perf_counter()
        _, inf2 = orc.cg(apply_a, rhs, tol=1e-10)
        conv["24^3x48_eo"] = {"seconds": round(time.perf_counter() - t0, 2), "iters": inf2["iters"],
                              "true_rel_resid": float("%.4g" % inf2["true_rel_resid"])}
        out["cg_to_convergence"] = conv
    return out


# ---------------------------------------------------------------------------------------------
# Oracle checks: the FP64 CPU oracle restates the residual of every reported solution (run after
# the timed region; the library never calls the oracle).  Reading C-7: an e/o CG stops on the
# normal-equation residual of the Schur system; solvers of D x = eta compared with each other stop
# on the system residual ||eta - D x|| / ||eta||.  Both are reported for every solve.
# ---------------------------------------------------------------------------------------------
def _norm(a):
    import numpy as np
    return float(np.sqrt(np.sum(np.abs(np.asarray(a)) ** 2)))


class OracleEo:
    """Restated residuals of e/o solves of D x = eta (x = (xe, xo) canonical halves):
    normal_eq = ||D_hat^+ bhat - D_hat^+ D_hat xe|| / ||D_hat^+ bhat||, system = ||eta - D x|| / ||eta||."""

    def __init__(self, u, kappa, ph, eta):
        from oracle import oracle as orc
        self.orc, self.u, self.kappa, self.ph, self.eta = orc, u, kappa, ph, eta
        self.dims = orc.dims_of(u)
        be, bo = orc.eo_split(eta, self.dims)
        bhat = orc.eo_prepare(be, bo, u, kappa, ph)
        self.rhs = orc.schur(bhat, u, kappa, ph, dagger=True)
        self.rhs_norm, self.eta_norm = _norm(self.rhs), _norm(eta)

    def check(self, xe, xo):
        orc, u, k, ph = self.orc, self.u, self.kappa, self.ph
        ax = orc.schur(orc.schur(xe, u, k, ph), u, k, ph, dagger=True)
        x = orc.eo_join(xe, xo, self.dims)
        return {"normal_eq": _norm(self.rhs - ax) / self.rhs_norm,
                "system": _norm(self.eta - orc.dirac(x, u, k, ph)) / self.eta_norm}


def oracle_full_residuals(u, kappa, ph, eta, x):
    """Restated residuals of a full-lattice solve of D x = eta: system = ||eta - D x|| / ||eta||,
    normal_eq = ||D^+ eta - D^+ D x|| / ||D^+ eta||."""
    from oracle import oracle as orc
    r = eta - orc.dirac(x, u, kappa, ph)
    rhs = orc.dirac(eta, u, kappa, ph, dagger=True)
    return {"system": _norm(r) / _norm(eta), "normal_eq": _norm(orc.dirac(r, u, kappa, ph, dagger=True)) / _norm(rhs)}


def summarize_checks(checks, tol=1e-10, key="normal_eq"):
    """checks: list of residual dicts; -> worst values and whether the criterion met tol (1 % slack
    for the last rounding of the restatement itself)."""
    worst = {k: max(c[k] for c in checks) for k in checks[0]}
    return {"worst": {k: float("%.4g" % v) for k, v in worst.items()}, "criterion": key,
            "criterion_met": bool(worst[key] <= tol * 1.01), "n": len(checks)}


def host_cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline leg")
    ap.add_argument("--no-extra", action="store_true",
                    help="default workload: skip the 32^3x64 mixed-precision and learned-preconditioner rows")
    ap.add_argument("--cpu-iters", type=int, default=25, help="CG iterations of the CPU-oracle sample")
    ap.add_argument("--cpu-quick", action="store_true",
                    help="skip the oracle CG-to-convergence runs of the CPU baseline")
    ap.add_argument("--workload", choices=["eo-cg", "mixed", "propagator", "learned", "batch", "eigcg", "access",
                                           "split", "launch"],
                    default="eo-cg",
                    help="eo-cg: the headline (24^3x48 FP64 e/o CG); mixed: 32^3x64 FP64 vs mixed-precision CG; "
                         "propagator: 12 point sources, multi-RHS vs sequential; learned: train the PTC "
                         "preconditioner on 16^3x32 fields and compare mixed-precision multi-RHS CG on the normal "
                         "equations of D M with plain FP64 CG on 32^3x64; "
                         "eigcg: a sequence of right-hand sides, incremental EigCG vs plain FP64 CG; "
                         "access: the link-spinor kernel with sequential, index-array and pointer addressing; "
                         "split: the bulk / boundary split half-dslash against the fused one; "
                         "launch: half-dslash launch-shape sweeps and plain device streams for reference")
    ap.add_argument("--eig-eps", type=float, default=0.8, help="eigcg: link roughness, U = exp(i eps H)")
    ap.add_argument("--eig-kappa", type=float, default=0.196, help="eigcg: hopping parameter")
    ap.add_argument("--eig-mu", type=float, default=0.0, help="eigcg: twisted mass")
    ap.add_argument("--eig-rhs", type=int, default=35, help="eigcg: right-hand sides in the sequence")
    ap.add_argument("--eig-collect", type=int, default=30, help="eigcg: right-hand sides that add vectors")
    ap.add_argument("--batch-sizes", choices=["uneven", "small"], default="uneven",
                    help="batch: 16^3x32 + 24^3x48 + 32^3x64 (uneven, each system fills the GPU) or "
                         "8^3x16 + 12^3x24 + 16^3x32 (small, none does)")
    ap.add_argument("--epochs", type=int, default=150, help="learned: training epochs")
    ap.add_argument("--learned-rhs", type=int, default=4, help="learned: Gaussian sources solved together")
    ap.add_argument("--train-fields", type=int, default=8, help="learned: number of 16^3x32 training fields")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MiB",
                    help="only run a plain device copy of this size (counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this benchmark runs on exactly one GPU (--gpus 1); %d requested" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py: no GPU available", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)

    if args.calibrate_copy:
        n = args.calibrate_copy << 20
        a = torch.empty(n, dtype=torch.uint8, device="cuda").fill_(1)
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": n, "launches": 5}))
        return

    if args.workload == "mixed":
        return run_mixed(args)
    if args.workload == "propagator":
        return run_propagator(args)
    if args.workload == "learned":
        return run_learned(args)
    if args.workload == "batch":
        return run_batch(args)
    if args.workload == "eigcg":
        return run_eigcg(args)
    if args.workload == "access":
        return run_access(args)
    if args.workload == "split":
        return run_split(args)
    if args.workload == "launch":
        return run_launch(args)
    return run_eo_cg(args)


class EoSolver:
    """One e/o solve of D x = eta on a context: prepare, D_hat^+, CG, reconstruct."""

    def __init__(self, lat, eta_full_internal, kappa, tol, nrhs=1):
        from paper_1405_0700_amd import wilson as W
        self.W, self.lat, self.kappa, self.nrhs = W, lat, kappa, nrhs
        B = eta_full_internal
        # an internal FULL field is the EVEN half followed by the ODD half
        self.Be, self.Bo = B[: B.numel() // 2], B[B.numel() // 2:]
        self.bhat = lat.new(W.WL_EVEN, W.WL_F64, nrhs)
        self.rhs = lat.new(W.WL_EVEN, W.WL_F64, nrhs)
        self.xe = lat.new(W.WL_EVEN, W.WL_F64, nrhs)
        self.xo = lat.new(W.WL_ODD, W.WL_F64, nrhs)
        self.params = W.wl_solver_params_default()
        self.params.tol = tol

    def set_precision(self, prec, recon):
        self.params.prec, self.params.recon = prec, recon

    def step(self):
        W, lat, k, n = self.W, self.lat, self.kappa, self.nrhs
        self.xe.zero_()
        W.wl_eo_prepare(lat.ctx, self.bhat, self.Be, self.Bo, k, nrhs=n)
        W.wl_dirac_apply(lat.ctx, self.rhs, self.bhat, W.WL_OP_DHAT, True, k, nrhs=n)
        st, info = W.wl_cg_solve(lat.ctx, self.xe, self.rhs, W.WL_OP_DHAT, k, nrhs=n, params=self.params)
        W.wl_eo_reconstruct(lat.ctx, self.xo, self.xe, self.Bo, k, nrhs=n)
        if st != W.WL_OK:
            print("[bench] solver status %d: %s" % (st, W.last_error()), file=sys.stderr)
        self.last_status = st
        return st, info

    def timed(self, steps, warmup):
        """-> (ms per step, infos of the last step)"""
        import torch
        for _ in range(warmup):
            self.step()
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        stream = torch.cuda.current_stream()
        ev0.record(stream)
        infos = []
        for _ in range(steps):
            infos.append(self.step()[1])
        ev1.record(stream)
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / steps, infos


# the same solve with other storage: FP64 with 12-real links (the third row rebuilt, exact up to rounding), then
# reduced-precision inner storage with FP64 reliable updates
MIXED = [("f64_12", 0, 12), ("f32_18", 1, 18), ("f32_12", 1, 12), ("f16n_12", 2, 12), ("bf16n_12", 3, 12),
         ("i16n_12", 4, 12)]


def run_config1(W):
    """The small cache-resident case: 8^4, links exp(0.5 i H) seed 101, Gaussian source seed 102, kappa
    0.12, full lattice: one full hopping term (both parities, FP64) and CG on the normal equations of D to
    ||eta - D x|| <= 1e-10 ||eta|| (wl_cgnr_solve), timed on the GPU and restated by the oracle.  The
    lattice fits in the caches: latency and parity, not an HBM measurement."""
    import torch
    from paper_1405_0700_amd import synth
    d1, kappa, ph = (8, 8, 8, 8), 0.12, WORKLOAD["phases"]
    u1 = synth.su3_links(d1, 0.5, 101)
    eta1 = synth.gaussian_spinor(d1, seed=102)
    lat = W.Lattice.create(u1, ph)
    try:
        b = lat.pack(eta1, W.WL_FULL)
        h = lat.new(W.WL_FULL)
        for _ in range(5):
            W.wl_dslash_apply(lat.ctx, h, b, W.WL_FULL)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(50):
            W.wl_dslash_apply(lat.ctx, h, b, W.WL_FULL)
        e1.record()
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) / 50 * 1e3
        x = lat.new(W.WL_FULL)
        W.wl_cgnr_solve(lat.ctx, x, b, kappa)  # warm-up (builds the solver's workspaces)
        x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, info = W.wl_cgnr_solve(lat.ctx, x, b, kappa)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        xs = lat.unpack(x, W.WL_FULL).reshape(eta1.shape)
    finally:
        lat.close()
    res = oracle_full_residuals(u1, kappa, ph, eta1, xs)
    return {"workload": "8^4, links exp(0.5iH) seed 101, Gaussian source seed 102, kappa 0.12, full D, FP64",
            "hopping_term_full_us": round(us, 2), "cg_normal_eq_ms": round(ms, 3), "iters": info["iters"],
            "status": st, "stopping_criterion": "||eta - D x|| <= 1e-10 ||eta|| (reading C-7)",
            "oracle": {k: float("%.4g" % v) for k, v in res.items()},
            "oracle_criterion_met": bool(res["system"] <= 1.01e-10)}


def run_launch(args):
    """Half-dslash launch shapes, timed with events over 20 back-to-back applications each, and plain device
    streams of 4 GiB for reference (what HBM gives a copy, a fill and a read here):
      f64_24 / f64_32   FP64-18 at 24^3x48 and 32^3x64 (links seed 401), two threads per point, over the
                        processing order (z-range depth -k, t-chunks k > 0, e/o order 0, y-z blocks YZ)
      f16n_32           FP16+norm-12 at 32^3x64: one or two threads per point, blocks, occupancy caps, orders
      rhs12_f32_24      12 right-hand sides FP32-18 at 24^3x48: one or two threads per point, time sweeps,
                        y-z blocks
      rhs12_f64_24      the same in FP64-18 (5,760 B per site), z-ranges against y-z blocks
    The library default of each context is listed first ("default")."""
    import torch
    from paper_1405_0700_amd import synth
    from paper_1405_0700_amd import wilson as W
    A, YZ = W.WL_TCHUNK_AUTO, W.WL_TCHUNK_YZ

    def timed(fn, n=20):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(n):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / n * 1e3

    n = 4 << 30
    a = torch.empty(n // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    hbm = {"copy_TBps": round(2 * n / timed(lambda: b.copy_(a), 10) / 1e6, 3),
           "fill_TBps": round(n / timed(lambda: b.fill_(2.0), 10) / 1e6, 3),
           "torch_sum_TBps": round(n / timed(lambda: a.sum(), 10) / 1e6, 3)}  # a reduction, not a bandwidth test
    del a, b
    torch.cuda.empty_cache()

    def sweep(dims, prec, recon, nrhs, site_bytes, cfgs):
        lat = W.Lattice.create(synth.su3_links(dims, 0.2, 401), (1, 1, 1, -1))
        vh = lat.volume // 2
        x = lat.new(W.WL_ODD, prec, nrhs)
        y = lat.new(W.WL_EVEN, prec, nrhs)
        src = lat.new(W.WL_ODD, W.WL_F32, nrhs)
        src.view(torch.float32).normal_(generator=torch.Generator(device="cuda").manual_seed(402))
        W.wl_convert_spinor(lat.ctx, x, prec, src, W.WL_F32, W.WL_ODD, nrhs)
        W.wl_ctx_prepare_links(lat.ctx, prec, recon)
        rows = []
        default = W.wl_ctx_get_launch(lat.ctx, prec)
        for name, cfg in [("default", default)] + [(None, c) for c in cfgs]:
            W.wl_ctx_set_launch(lat.ctx, prec, *cfg)
            us = timed(lambda: W.wl_dslash_apply(lat.ctx, y, x, W.WL_EVEN, prec, recon, nrhs))
            rows.append({"launch": list(cfg), "us": round(us, 2),
                         "algorithmic_GBps": round(site_bytes * vh / us / 1e3, 1)} | ({"default": True} if name else {}))
        lat.close()
        return rows

    cfg = lambda block, tps, tch, occ=0, sweep_=0: (block, 1, tps, tch, -1, 1, occ, sweep_)
    out = {
        "f64_24": sweep((24, 24, 24, 48), W.WL_F64, 18, 1, 1536,
                        [cfg(128, 2, t) for t in (-3, -6, -12, 0, 4, YZ)]),
        "f64_32": sweep((32, 32, 32, 64), W.WL_F64, 18, 1, 1536,
                        [cfg(128, 2, t) for t in (-4, -8, 0, 8, YZ)]),
        "f16n_32": sweep((32, 32, 32, 64), W.WL_F16N, 12, 1, 296,
                         [cfg(bl, tps, A, occ) for tps in (1, 2) for bl in (128, 256) for occ in (0, 4)]
                         + [cfg(256, 1, YZ, 4), cfg(256, 1, 0, 4)]),
        "rhs12_f32_24": sweep((24, 24, 24, 48), W.WL_F32, 18, 12, 2880,
                              [cfg(256, 2, A), cfg(256, 1, A)] + [cfg(256, 1, 0, 0, sw) for sw in (4, 8, 16)]
                              + [cfg(bl, tps, YZ) for tps in (1, 2) for bl in (128, 256)]),
        "rhs12_f64_24": sweep((24, 24, 24, 48), W.WL_F64, 18, 12, 1152 + 2 * 2304,
                              [cfg(bl, tps, t) for t in (A, YZ) for tps in (1, 2) for bl in (128, 256)]),
    }
    print(json.dumps({"metric": "half-dslash time per launch shape (us), algorithmic GB/s; device streams (TB/s)",
                      "unit": "us", "higher_is_better": False, "workload": "launch", "hbm_streams_4GiB": hbm,
                      "sweeps": out}))


def run_eo_cg(args):
    import torch
    from paper_1405_0700_amd import wilson as W
    wl = WORKLOAD
    t0 = time.perf_counter()
    u, eta = make_inputs(wl)
    print("[bench] inputs generated in %.1f s" % (time.perf_counter() - t0), file=sys.stderr, flush=True)
    lat = W.Lattice.create(u, wl["phases"])
    vh = lat.volume // 2
    kappa = wl["kappa"]
    solver = EoSolver(lat, lat.pack(eta, W.WL_FULL), kappa, wl["tol"])

    for _ in range(args.warmup):
        solver.step()
    torch.cuda.synchronize()
    # every 5th hopping launch (5 is coprime to the 4 launches of an iteration, so every
    # kind is sampled) carries a pair of HIP events: the live kernel timing for the
    # roofline, at a fifth of the instrumentation's cost to the timed step
    W.wl_timing_enable(lat.ctx, True, every=5)
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    infos = []
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(args.steps):
        st, info = solver.step()
        infos.append(info[0])
    ev1.record(stream)
    torch.cuda.synchronize()
    total_ms = ev0.elapsed_time(ev1)
    ms_per_step = total_ms / args.steps
    nbytes = sum(step_bytes(vh, i["iters"], i["restarts"]) for i in infos)
    value = nbytes / (total_ms * 1e-3) / 1e9

    n_hop, ms_hop = W.wl_timing_read(lat.ctx, W.WL_F64, 18, False, 0)
    W.wl_timing_enable(lat.ctx, False)
    avg_ms = ms_hop / max(n_hop, 1)
    achieved = SITE_BYTES["hop"] * vh / (avg_ms * 1e-3) / 1e9
    traffic = read_traffic()
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": "wl::hop_kernel_split<0, 0, 18, false, 16, true> (FP64 half-dslash H_oe, 18-real links, non-temporal link loads, output through the caches)",
                "launches": n_hop, "avg_us": round(avg_ms * 1e3, 2),
                "algorithmic_bytes_per_launch": SITE_BYTES["hop"] * vh}
    sols = {"f64_18": (lat.unpack(solver.xe, W.WL_EVEN), lat.unpack(solver.xo, W.WL_ODD))}

    # the same solve with reduced-precision storage (time to the same FP64 tolerance)
    mixed = {}
    for name, prec, recon in MIXED:
        solver.set_precision(prec, recon)
        ms, inf = solver.timed(args.steps, 1)
        mixed[name] = {"time_to_solution_ms": round(ms, 3), "iters": inf[-1][0]["iters"],
                       "status": solver.last_status, "reliable_updates": inf[-1][0]["reliable_updates"],
                       "true_rel_resid_gpu": inf[-1][0]["true_rel_resid"],
                       "speedup_vs_f64": round(ms_per_step / ms, 3)}
        sols[name] = (lat.unpack(solver.xe, W.WL_EVEN), lat.unpack(solver.xo, W.WL_ODD))

    # the oracle restates every solution's residuals (after the timed region)
    check = OracleEo(u, kappa, wl["phases"], eta)
    head = check.check(*sols["f64_18"])
    for name in mixed:
        mixed[name]["oracle"] = {k: float("%.4g" % v) for k, v in check.check(*sols[name]).items()}
    config1 = run_config1(W)
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(u, eta, wl, args.cpu_iters, converge=not args.cpu_quick)
    extra = {} if args.no_extra else extra_rows(args)

    last = infos[-1]
    line = {
        "metric": "dslash GB/s (% HBM peak); CG time-to-1e-10: plain FP64 vs mixed/learned",
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "even/odd Wilson CG to 1e-10, 24^3x48, kappa 0.135, links exp(0.2iH) seed 201, "
                               "Gaussian source seed 202, FP64, 18-real links",
                   "lattice": list(wl["dims"]), "kappa": kappa, "precision": "f64", "recon": 18},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "time_to_solution_ms": round(ms_per_step, 3),
        "cg_iters": last["iters"],
        "cg_restarts": last["restarts"],
        "cg_status": st,
        "stopping_criterion": "||D_hat^+ bhat - D_hat^+ D_hat x_e|| <= 1e-10 ||D_hat^+ bhat|| (CG on the normal "
                              "equations of the Schur system)",
        "true_rel_resid_gpu": last["true_rel_resid"],
        "oracle_normal_eq_rel_resid": float("%.4g" % head["normal_eq"]),
        "oracle_full_system_rel_resid": float("%.4g" % head["system"]),
        "oracle_criterion_met": bool(head["normal_eq"] <= wl["tol"] * 1.01),
        "algorithmic_bytes_per_step": nbytes // args.steps,
        "mixed_precision_same_system": mixed,
        "config1_8x8x8x8": config1,
    } | extra
    print(json.dumps(line))
    lat.close()


def extra_rows(args):
    """The 32^3x64 rows of the line (after the timed region): FP64 CG against FP16+norm and BF16+norm
    mixed CG (the mixed workload's system, one timed solve each), and the learned preconditioner
    (trained as in the learned workload, tested on the same 32^3x64 field with 2 Gaussian sources)
    against plain FP64 CGNR; the oracle restates every solution."""
    log = lambda m: print("[bench] " + m, file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    u, eta = make_inputs(MIXED_32)
    log("32^3x64 inputs in %.1f s" % (time.perf_counter() - t0))
    sub = argparse.Namespace(**vars(args))
    sub.steps, sub.warmup = 1, 1
    res, ok = mixed_results(sub, u, eta, [("f64_18", 0, 18), ("f16n_12", 2, 12), ("bf16n_12", 3, 12)])
    mixed = {"workload": "even/odd Wilson CG to 1e-10, 32^3x64, kappa 0.137, links exp(0.2iH) seed 301, source "
                         "seed 302 (1 warm-up + 1 timed solve per format)",
             "results": {k: {"time_to_solution_ms": v["time_to_solution_ms"], "iters": v["iters"],
                             "status": v["status"], "oracle": v["oracle"]} for k, v in res.items()},
             "oracle_check": ok,
             "speedup_vs_f64": {k: round(res["f64_18"]["time_to_solution_ms"] / v["time_to_solution_ms"], 3)
                                for k, v in res.items() if k != "f64_18"}}
    learned = learned_results(args, u_test=u, test_seed=None, src_seeds=(311, 312),
                              solvers=("cg_f64", "pcgnr_none", "pcgnr_trained"))
    learned = {k: learned[k] for k in ("workload", "stopping_criterion", "epochs", "loss_first", "loss_last",
                                       "results", "network_apply_ms", "speedup_per_source_vs_cg_f64")}
    log("32^3x64 rows in %.1f s" % (time.perf_counter() - t0))
    return {"config3_mixed_32x32x32x64": mixed, "config5_learned_32x32x32x64": learned}


MIXED_32 = dict(dims=(32, 32, 32, 64), eps=0.2, gauge_seed=301, src_seed=302, kappa=0.137, phases=(1, 1, 1, -1),
                tol=1e-10)


def mixed_results(args, u, eta, formats):
    """FP64 CG against mixed-precision CG (FP64 reliable updates) on the 32^3x64 system of MIXED_32
    (links u, source eta), every solution restated by the oracle; -> (results, oracle summary)."""
    from paper_1405_0700_amd import wilson as W
    wl = MIXED_32
    lat = W.Lattice.create(u, wl["phases"])
    solver = EoSolver(lat, lat.pack(eta, W.WL_FULL), wl["kappa"], wl["tol"])
    res, sols = {}, {}
    for name, prec, recon in formats:
        solver.set_precision(prec, recon)
        ms, inf = solver.timed(args.steps, args.warmup)
        res[name] = {"time_to_solution_ms": round(ms, 3), "iters": inf[-1][0]["iters"],
                     "status": solver.last_status, "reliable_updates": inf[-1][0]["reliable_updates"],
                     "restarts": inf[-1][0]["restarts"], "true_rel_resid_gpu": inf[-1][0]["true_rel_resid"]}
        sols[name] = (lat.unpack(solver.xe, W.WL_EVEN), lat.unpack(solver.xo, W.WL_ODD))
        print("[bench] %s %s" % (name, res[name]), file=sys.stderr, flush=True)
    lat.close()
    # the oracle restates every solution (normal-equation criterion and full system)
    check = OracleEo(u, wl["kappa"], wl["phases"], eta)
    for name in res:
        res[name]["oracle"] = {k: float("%.4g" % v) for k, v in check.check(*sols[name]).items()}
        print("[bench] oracle %s %s" % (name, res[name]["oracle"]), file=sys.stderr, flush=True)
    return res, summarize_checks([r["oracle"] for r in res.values()])


def run_mixed(args):
    """32^3x64, kappa 0.137: FP64 CG against mixed-precision CG (FP64 reliable updates)."""
    u, eta = make_inputs(MIXED_32)
    res, ok = mixed_results(args, u, eta, [("f64_18", 0, 18)] + MIXED)
    best = min((v["time_to_solution_ms"], k) for k, v in res.items() if k != "f64_18")
    print(json.dumps({"metric": "CG time-to-1e-10, plain FP64 vs mixed precision", "workload":
                      "even/odd Wilson CG, 32^3x64, kappa 0.137, links exp(0.2iH) seed 301, source seed 302",
                      "stopping_criterion": "normal equations of the Schur system, 1e-10 (reading C-7)",
                      "unit": "ms", "higher_is_better": False, "results": res, "oracle_check": ok,
                      "best_mixed": best[1], "speedup_best_mixed_vs_f64": round(res["f64_18"]["time_to_solution_ms"] / best[0], 3)}))


def run_propagator(args):
    """24^3x48, kappa 0.135: the 12 spin-colour point sources at the origin, solved one by
    one and together in one multi-RHS solve; plus the multi-RHS dslash throughput."""
    import numpy as np
    import torch
    from paper_1405_0700_amd import synth
    from paper_1405_0700_amd import wilson as W
    dims, kappa = (24, 24, 24, 48), 0.135
    u = synth.su3_links(dims, 0.2, 401)
    lat = W.Lattice.create(u, (1, 1, 1, -1))
    vh = lat.volume // 2
    etas = np.stack([synth.point_source(dims, s, c).reshape(-1, 4, 3) for s in range(4) for c in range(3)])
    res, sols = {}, {}
    for name, prec, recon in [("f64_18", 0, 18), ("f32_18", 1, 18), ("f16n_12", 2, 12)]:
        multi = EoSolver(lat, lat.pack(etas, W.WL_FULL, W.WL_F64, 12), kappa, 1e-10, nrhs=12)
        multi.set_precision(prec, recon)
        ms_multi, inf = multi.timed(args.steps, args.warmup)
        iters = [i["iters"] for i in inf[-1]]
        status_multi = multi.last_status
        sols[name] = {"multi": (lat.unpack(multi.xe, W.WL_EVEN, W.WL_F64, 12),
                                lat.unpack(multi.xo, W.WL_ODD, W.WL_F64, 12))}
        singles = [EoSolver(lat, lat.pack(etas[k], W.WL_FULL), kappa, 1e-10) for k in range(12)]
        for s_ in singles:
            s_.set_precision(prec, recon)
        def all12():
            for s_ in singles:
                s_.step()
        for _ in range(args.warmup):
            all12()
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(args.steps):
            all12()
        ev1.record()
        torch.cuda.synchronize()
        ms_seq = ev0.elapsed_time(ev1) / args.steps
        sols[name]["sequential"] = [(lat.unpack(s_.xe, W.WL_EVEN), lat.unpack(s_.xo, W.WL_ODD)) for s_ in singles]
        res[name] = {"twelve_rhs_one_solve_ms": round(ms_multi, 3), "twelve_sequential_solves_ms": round(ms_seq, 3),
                     "speedup": round(ms_seq / ms_multi, 3), "iters": iters, "status_multi": status_multi,
                     "status_sequential": [s_.last_status for s_ in singles]}
        print("[bench] %s %s" % (name, res[name]), file=sys.stderr, flush=True)
        del multi, singles
    # 12-RHS half-dslash throughput (FP32 storage, 18-real links): 576 B of links + 12 x 192 B of spinors per site
    x = lat.new(W.WL_ODD, W.WL_F32, 12)
    y = lat.new(W.WL_EVEN, W.WL_F32, 12)

    def dslash12_us():
        for _ in range(3):
            W.wl_dslash_apply(lat.ctx, y, x, W.WL_EVEN, W.WL_F32, 18, 12)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(20):
            W.wl_dslash_apply(lat.ctx, y, x, W.WL_EVEN, W.WL_F32, 18, 12)
        ev1.record()
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / 20 * 1e3

    # the library's default launch shape, then the one the autotuner picks for 12 right-hand sides
    us_default = dslash12_us()
    tuned_cfg, _, _ = W.wl_autotune(lat.ctx, W.WL_F32, 18, 12)
    us = dslash12_us()
    gbs = (576 + 12 * 192) * vh / us / 1e3
    lat.close()
    # the oracle restates all 12 sources of every solve (multi-RHS and sequential)
    for k in range(12):
        check = OracleEo(u, kappa, (1, 1, 1, -1), etas[k].reshape(u.shape[:4] + (4, 3)))
        for name in res:
            xe, xo = sols[name]["multi"]
            res[name].setdefault("oracle_multi", []).append(check.check(xe[k], xo[k]))
            res[name].setdefault("oracle_sequential", []).append(check.check(*sols[name]["sequential"][k]))
        print("[bench] oracle source %d done" % k, file=sys.stderr, flush=True)
    for name in res:
        res[name]["oracle_multi"] = summarize_checks(res[name]["oracle_multi"])
        res[name]["oracle_sequential"] = summarize_checks(res[name]["oracle_sequential"])
    print(json.dumps({"metric": "12-RHS propagator: one multi-RHS solve vs 12 solves", "unit": "ms",
                      "workload": "24^3x48, kappa 0.135, links exp(0.2iH) seed 401, 12 point sources at the origin",
                      "stopping_criterion": "normal equations of the Schur system, 1e-10 per source (reading C-7)",
                      "higher_is_better": False, "results": res,
                      "dslash_12rhs_f32_18": {"us": round(us, 2), "algorithmic_GBps": round(gbs, 1),
                                               "launch": list(tuned_cfg), "us_default_launch": round(us_default, 2),
                                               "bytes_per_site": 576 + 12 * 192}}))


def run_batch(args):
    """Uneven batch: 16^3x32, 24^3x48 and 32^3x64 (links exp(0.2iH), seeds 411-413), 4 Gaussian
    right-hand sides each (seeds 421-423), kappa 0.135, e/o CG on the normal equations to 1e-10,
    FP32 inner with FP64 reliable updates and a graph-captured iteration: all three systems in
    one batched solve (one persistent launch per hopping stage; then the autotuned launch, which
    may be one launch per system; then one launch per system) vs the three solved one after
    another; plus the persistent D_hat launch over all three against three separate launches."""
    import numpy as np
    import torch
    from paper_1405_0700_amd import synth
    from paper_1405_0700_amd import wilson as W
    kappa, nrhs, ph = 0.135, 4, (1, 1, 1, -1)
    sysdims = [(16, 16, 16, 32), (24, 24, 24, 48), (32, 32, 32, 64)]
    if args.batch_sizes == "small":
        sysdims = [(8, 8, 8, 16), (12, 12, 12, 24), (16, 16, 16, 32)]
    log = lambda m: print("[bench] " + m, file=sys.stderr, flush=True)
    lats, etas, us_, stacks = [], [], [], []
    for k, dims in enumerate(sysdims):
        us_.append(synth.su3_links(dims, 0.2, 411 + k))
        lats.append(W.Lattice.create(us_[-1], ph))
        stack = np.stack([synth.gaussian_spinor(dims, seed=1000 * (421 + k) + r) for r in range(nrhs)])
        stacks.append(stack)
        etas.append(lats[-1].pack(stack.reshape(nrhs, -1, 4, 3), W.WL_FULL, W.WL_F64, nrhs))
    log("inputs ready")
    batch = W.wl_batch_create([l.ctx for l in lats])
    singles = [EoSolver(l, e, kappa, 1e-10, nrhs=nrhs) for l, e in zip(lats, etas)]
    for s_ in singles:
        s_.set_precision(W.WL_F32, 18)
        s_.params.use_graph = 1
    params = W.wl_solver_params_default()
    params.prec, params.recon, params.use_graph, params.tol = W.WL_F32, 18, 1, 1e-10

    def batched():
        for s_ in singles:
            s_.xe.zero_()
            W.wl_eo_prepare(s_.lat.ctx, s_.bhat, s_.Be, s_.Bo, kappa, nrhs=nrhs)
            W.wl_dirac_apply(s_.lat.ctx, s_.rhs, s_.bhat, W.WL_OP_DHAT, True, kappa, nrhs=nrhs)
        st, info = W.wl_batch_cg_solve(batch, [s_.xe for s_ in singles], [s_.rhs for s_ in singles],
                                       W.WL_OP_DHAT, [kappa] * 3, nrhs, params)
        for s_ in singles:
            W.wl_eo_reconstruct(s_.lat.ctx, s_.xo, s_.xe, s_.Bo, kappa, nrhs=nrhs)
        return st, info

    def sequential():
        return [s_.step() for s_ in singles]

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.steps):
            out = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) * 1e3 / args.steps, out

    def solutions():
        """the current solutions (every system and rhs) as canonical halves, for the oracle check"""
        return [(s_.lat.unpack(s_.xe, W.WL_EVEN, W.WL_F64, nrhs), s_.lat.unpack(s_.xo, W.WL_ODD, W.WL_F64, nrhs))
                for s_ in singles]

    res, sols = {}, {}
    ms_seq, out_seq = timed(sequential)
    res["sequential_ms"] = round(ms_seq, 2)
    res["sequential_iters"] = [[i["iters"] for i in info] for _, info in out_seq]
    res["sequential_status"] = [st_ for st_, _ in out_seq]
    sols["sequential"] = solutions()
    log("sequential %.1f ms" % ms_seq)
    default_launch = W.wl_batch_get_launch(batch)
    ms_b, (st, info) = timed(batched)
    res["batched_default_ms"] = round(ms_b, 2)
    res["batched_default_launch"] = default_launch
    res["batched_iters"] = [[i["iters"] for i in s] for s in info]
    res["batched_default_status"] = st
    sols["batched_default"] = solutions()
    log("batched (default launch %s) %.1f ms" % (default_launch, ms_b))
    tuned, tuned_us, _ = W.wl_batch_autotune(batch, W.WL_F32, 18, nrhs)
    ms_t, (st, _) = timed(batched)
    res["batched_tuned_ms"] = round(ms_t, 2)
    res["batched_tuned_launch"] = tuned
    res["batched_tuned_status"] = st
    sols["batched_tuned"] = solutions()
    log("batched (tuned launch %s) %.1f ms" % (tuned, ms_t))
    # lockstep with one launch per system and stage (workgroups 0)
    W.wl_batch_set_launch(batch, 0, *default_launch[1:])
    ms_p, (st, info) = timed(batched)
    res["batched_per_system_launches_ms"] = round(ms_p, 2)
    res["batched_per_system_status"] = st
    sols["batched_per_system"] = solutions()
    log("batched (per-system launches) %.1f ms" % ms_p)
    W.wl_batch_set_launch(batch, *default_launch)
    # the persistent D_hat over all three systems against three separate D_hat applications
    ins = [l.new(W.WL_EVEN, W.WL_F32, nrhs) for l in lats]
    for t_ in ins:
        t_.copy_(torch.zeros_like(t_))
    outs = [l.new(W.WL_EVEN, W.WL_F32, nrhs) for l in lats]
    vhs = [l.volume // 2 for l in lats]
    bytes_apply = sum(v * (2 * 576 + nrhs * (192 + 288)) for v in vhs)

    def persistent():
        W.wl_batch_dirac_apply(batch, outs, ins, W.WL_OP_DHAT, False, [kappa] * 3, W.WL_F32, 18, nrhs)

    def separate():
        for l, o, i_ in zip(lats, outs, ins):
            W.wl_dirac_apply(l.ctx, o, i_, W.WL_OP_DHAT, False, kappa, W.WL_F32, 18, nrhs)

    for name, fn in (("persistent", persistent), ("separate", separate)):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(20):
            fn()
        e1.record()
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) / 20 * 1e3
        res["dhat_apply_" + name] = {"us": round(us, 2), "algorithmic_GBps": round(bytes_apply / us / 1e3, 1)}
        log("%s D_hat over the three systems: %.1f us" % (name, us))
    res["dhat_apply_bytes"] = bytes_apply
    W.wl_batch_destroy(batch)
    batch = None
    # the oracle restates every system and rhs of every variant
    checks = {k: [] for k in sols}
    for sy in range(len(sysdims)):
        for r in range(nrhs):
            check = OracleEo(us_[sy], kappa, ph, stacks[sy][r])
            for k in sols:
                xe, xo = sols[k][sy]
                checks[k].append(check.check(xe[r], xo[r]))
        log("oracle system %d done" % sy)
    res["oracle"] = {k: summarize_checks(v) for k, v in checks.items()}
    names = " + ".join("%d^3x%d" % (d[0], d[3]) for d in sysdims)
    print(json.dumps({"metric": "uneven batch (%s, 4 RHS each): batched vs sequential time-to-1e-10" % names,
                      "unit": "ms", "higher_is_better": False, "kappa": kappa,
                      "precision": "FP32 inner, FP64 reliable updates, graph-captured iteration",
                      "stopping_criterion": "normal equations of each Schur system, 1e-10 per rhs (reading C-7)",
                      "results": res, "speedup_tuned_vs_sequential": round(ms_seq / ms_t, 3)}))


LEARNED_ALL = ("cg_f64", "cg_f64_multi", "pcgnr_none", "pcgnr_trained", "pcgnr_initial", "fgcr_none", "fgcr_trained")


def run_learned(args):
    out = learned_results(args)
    print(json.dumps(out))


def learned_results(args, u_test=None, test_seed=520, src_seeds=None, solvers=LEARNED_ALL):
    """Config 5: train the PTC preconditioner (8 hidden channels, BF16 weights) with the library's own
    kernels on (source, solution) pairs from plain FP64 CG on 8 fields 16^3x32 (kappa 0.137, links
    exp(0.2iH) seeds 501-508, 4 Gaussian sources each, residual-norm loss), then solve
    D x = eta on 32^3x64 (links seed 520) for `--learned-rhs` Gaussian sources (seeds 521...), every
    solver stopped on ||eta - D x|| <= 1e-10 ||eta|| (reading C-7):
      cg_f64            plain FP64 CGNR, one source after another (the comparison of the benchmark spec)
      cg_f64_multi      plain FP64 CGNR, all sources in one multi-RHS solve
      pcgnr_none        mixed precision (FP32 inner, FP64 defect correction), multi-RHS, no network
      pcgnr_initial     the same with the untrained network
      pcgnr_trained     the same with the trained network
      fgcr_none         flexible GCR (FP64), one source after another, no network
      fgcr_trained      the same with the trained network as right preconditioner
    The oracle restates every source's residual.  u_test / src_seeds replace the test field and the
    sources' seeds (the default line reuses the mixed workload's 32^3x64 field); `solvers` picks rows."""
    import numpy as np
    import torch
    from paper_1405_0700_amd import learned, synth
    from paper_1405_0700_amd import wilson as W
    kappa, ph, nsrc = 0.137, (1, 1, 1, -1), args.learned_rhs
    log = lambda m: print("[bench] " + m, file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    sets = []
    for k in range(args.train_fields):
        dims = (16, 16, 16, 32)
        lat = W.Lattice.create(synth.su3_links(dims, 0.2, 501 + k), ph)
        srcs = [synth.gaussian_spinor(dims, seed=1000 * (511 + k) + j) for j in range(4)]
        sets.append((lat, learned.harvest(lat, srcs, kappa)))
    torch.cuda.synchronize()
    t_harvest = time.perf_counter() - t0
    log("harvested %d pairs in %.1f s" % (sum(len(p) for _, p in sets), t_harvest))
    w1, w2 = synth.ptc_weights(8, 530)
    net = W.wl_ptc_create(w1, w2)
    t0 = time.perf_counter()
    losses = learned.train(sets, net, args.epochs, lr=1e-3, log=log, loss="residual", kappa=kappa)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    for lat_, _ in sets:
        lat_.close()
    dims = (32, 32, 32, 64)
    if u_test is None:
        u_test = synth.su3_links(dims, 0.2, test_seed)
    src_seeds = list(src_seeds) if src_seeds is not None else [test_seed + 1 + k for k in range(nsrc)]
    nsrc = len(src_seeds)
    etas = [synth.gaussian_spinor(dims, seed=sd) for sd in src_seeds]
    lat = W.Lattice.create(u_test, ph)
    eta_m = lat.pack(np.stack([e.reshape(-1, 4, 3) for e in etas]), W.WL_FULL, W.WL_F64, nsrc)
    eta_1 = [lat.pack(e, W.WL_FULL) for e in etas]
    fresh = W.wl_ptc_create(w1, w2)
    res, sols = {}, {}

    def timed(fn):
        torch.cuda.synchronize()
        t = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        return out, (time.perf_counter() - t) * 1e3

    # plain FP64 CGNR, one source at a time
    xs, its, sts, total = [], [], [], 0.0
    for k in range(nsrc if "cg_f64" in solvers else 0):
        x = lat.new(W.WL_FULL)
        (st, info), ms = timed(lambda: W.wl_cgnr_solve(lat.ctx, x, eta_1[k], kappa))
        total += ms
        xs.append(lat.unpack(x, W.WL_FULL))
        its.append(info["iters"])
        sts.append(st)
    if "cg_f64" in solvers:
        res["cg_f64"] = {"status": sts, "time_ms": round(total, 2), "time_per_source_ms": round(total / nsrc, 2),
                         "iters": its}
        sols["cg_f64"] = xs
        log("cg_f64 %s" % res["cg_f64"])
    if "cg_f64_multi" in solvers:
        x = lat.new(W.WL_FULL, W.WL_F64, nsrc)
        (st, infos), ms = timed(lambda: W.wl_cgnr_solve(lat.ctx, x, eta_m, kappa, nrhs=nsrc))
        infos = infos if nsrc > 1 else [infos]
        res["cg_f64_multi"] = {"status": st, "time_ms": round(ms, 2), "time_per_source_ms": round(ms / nsrc, 2),
                               "iters": [i["iters"] for i in infos]}
        sols["cg_f64_multi"] = list(lat.unpack(x, W.WL_FULL, W.WL_F64, nsrc).reshape(nsrc, -1, 4, 3))
        log("cg_f64_multi %s" % res["cg_f64_multi"])
    for name, m in (("pcgnr_none", None), ("pcgnr_trained", net), ("pcgnr_initial", fresh)):
        if name not in solvers:
            continue
        x = lat.new(W.WL_FULL, W.WL_F64, nsrc)
        pp = W.wl_pcgnr_params_default()
        pp.maxiter = 3000
        (st, infos), ms = timed(lambda: W.wl_pcgnr_solve(lat.ctx, x, eta_m, kappa, m, pp, nrhs=nsrc))
        infos = infos if nsrc > 1 else [infos]
        res[name] = {"status": st, "time_ms": round(ms, 2), "time_per_source_ms": round(ms / nsrc, 2),
                     "iters": [i["iters"] for i in infos], "cycles": [i["restarts"] for i in infos],
                     "fallback": [i["fallback"] for i in infos]}
        sols[name] = list(lat.unpack(x, W.WL_FULL, W.WL_F64, nsrc).reshape(nsrc, -1, 4, 3))
        log("%s %s" % (name, res[name]))
    # FGCR with the network as right preconditioner (one application per iteration), one source at a time
    for name, m in (("fgcr_none", None), ("fgcr_trained", net)):
        if name not in solvers:
            continue
        xs, its, sts, fbs, total = [], [], [], [], 0.0
        for k in range(nsrc):
            x = lat.new(W.WL_FULL)
            pf = W.wl_fgcr_params_default()
            pf.maxiter = 3000
            (st, info), ms = timed(lambda: W.wl_fgcr_solve(lat.ctx, x, eta_1[k], kappa, m, pf))
            total += ms
            xs.append(lat.unpack(x, W.WL_FULL))
            its.append(info["iters"])
            sts.append(st)
            fbs.append(info["fallback"])
        res[name] = {"status": sts, "time_ms": round(total, 2), "time_per_source_ms": round(total / nsrc, 2),
                     "iters": its, "fallback": fbs}
        sols[name] = xs
        log("%s %s" % (name, res[name]))
    # cost of one network application at this size (nsrc right-hand sides, forward)
    a = lat.new(W.WL_FULL, W.WL_F32, nsrc)
    b = lat.new(W.WL_FULL, W.WL_F32, nsrc)
    (_, ms_net) = timed(lambda: [W.wl_ptc_apply(lat.ctx, net, b, a, nrhs=nsrc) for _ in range(10)])
    lat.close()
    # the oracle restates every source of every solver (system criterion, reading C-7)
    for name in res:
        checks = [oracle_full_residuals(u_test, kappa, ph, etas[k], np.asarray(sols[name][k]).reshape(etas[k].shape))
                  for k in range(nsrc)]
        res[name]["oracle"] = summarize_checks(checks, key="system")
        log("oracle %s %s" % (name, res[name]["oracle"]))
    base = res["cg_f64"]["time_per_source_ms"]
    W.wl_ptc_destroy(net)
    W.wl_ptc_destroy(fresh)
    field = "links seed %d" % test_seed if test_seed is not None else "the mixed workload's links (seed 301)"
    return {"metric": "time-to-1e-10 of D x = eta: mixed-precision multi-RHS CG on the normal equations "
                      "of D M with the learned PTC preconditioner M vs plain FP64 CG",
            "unit": "ms", "higher_is_better": False,
            "workload": "train %d x 16^3x32 (links seeds 501-%d, 4 Gaussian sources each, pairs (source, "
                        "solution)), kappa 0.137; test 32^3x64 %s, %d sources (seeds %s)"
                        % (args.train_fields, 500 + args.train_fields, field, nsrc,
                           ", ".join(str(sd) for sd in src_seeds)),
            "stopping_criterion": "||eta - D x|| <= 1e-10 ||eta|| for every solver and source (reading C-7)",
            "harvest_s": round(t_harvest, 2), "train_s": round(t_train, 2), "epochs": args.epochs,
            "loss_first": losses[0], "loss_last": losses[-1], "results": res,
            "network_apply_ms": round(ms_net / 10, 3),
            "speedup_per_source_vs_cg_f64": {k: round(base / v["time_per_source_ms"], 3)
                                             for k, v in res.items() if k != "cg_f64"}}


def run_eigcg(args):
    """A sequence of right-hand sides of A = D_hat^+ D_hat (optionally twisted) on 24^3x48,
    links exp(i eps H) seed 402 (default eps 0.8 with kappa 0.196, near this field's
    critical kappa, where D_hat has small singular values and plain CG needs several
    hundred iterations), Gaussian sources on the even sites (seeds 440...), all to
    ||b - A x|| <= 1e-8 ||b|| in FP64: plain CG (the library's captured FP64 CG) per
    right-hand side against incremental EigCG with nev = 10, m = 60, up to 300 vectors,
    collecting on the first `eig_collect` right-hand sides (the paper's protocol for its
    35 right-hand sides)."""
    import torch
    from paper_1405_0700_amd import synth
    from paper_1405_0700_amd import wilson as W
    dims, tol = (24, 24, 24, 48), 1e-8
    kappa, mu, nrhs, ncol = args.eig_kappa, args.eig_mu, args.eig_rhs, args.eig_collect
    log = lambda m: print("[bench] " + m, file=sys.stderr, flush=True)
    lat = W.Lattice.create(synth.su3_links(dims, args.eig_eps, 402), (1, 1, 1, -1))
    bs = [lat.pack(synth.gaussian_spinor(dims, seed=440 + k, nsites=lat.volume // 2), W.WL_EVEN)
          for k in range(nrhs)]
    x = lat.new(W.WL_EVEN)
    p = W.wl_solver_params_default()
    p.tol, p.mu, p.maxiter = tol, mu, 100000

    def cg(b):
        x.zero_()
        return W.wl_cg_solve(lat.ctx, x, b, W.WL_OP_DHAT, kappa, params=p)

    cg(bs[0])  # warm-up: builds the FP64 links and captures the iteration graph
    torch.cuda.synchronize()
    cg_ms, cg_it = [], []
    for b in bs:
        t = time.perf_counter()
        st, info = cg(b)
        torch.cuda.synchronize()
        cg_ms.append((time.perf_counter() - t) * 1e3)
        cg_it.append(info[0]["iters"])
        if st != W.WL_OK:
            log("cg status %d" % st)
    log("cg iterations %s, %.1f ms total" % (cg_it, sum(cg_ms)))
    e = W.wl_eigcg_create(lat.ctx, W.WL_OP_DHAT, kappa, mu, 10, 60, 300)
    eig_ms, eig_it, eig_res = [], [], []
    for k, b in enumerate(bs):
        t = time.perf_counter()
        st, info = W.wl_eigcg_solve(e, x, b, tol=tol, collect=k < ncol)
        eig_ms.append((time.perf_counter() - t) * 1e3)
        eig_it.append(info["iters"])
        eig_res.append(info["true_rel_resid"])
        if st != W.WL_OK:
            log("eigcg status %d" % st)
        log("eigcg rhs %d: %d iterations, %.1f ms, %d vectors" % (k, info["iters"], eig_ms[-1],
                                                                 len(W.wl_eigcg_vectors(e, 300))))
    ritz = W.wl_eigcg_vectors(e, 300)
    W.wl_eigcg_destroy(e)
    # the same sequence with EigCG's own CG loop and no deflation: its per-iteration cost
    e0 = W.wl_eigcg_create(lat.ctx, W.WL_OP_DHAT, kappa, mu, 10, 60, 0)
    t = time.perf_counter()
    _, info0 = W.wl_eigcg_solve(e0, x, bs[0], tol=tol, collect=False)
    plain_loop_ms = (time.perf_counter() - t) * 1e3
    W.wl_eigcg_destroy(e0)
    tail = slice(ncol, nrhs)
    print(json.dumps({
        "metric": "time for a sequence of right-hand sides: incremental EigCG vs plain FP64 CG", "unit": "ms",
        "higher_is_better": False,
        "workload": "24^3x48, links exp(%g iH) seed 402, kappa %g, mu %g, %d Gaussian even-site sources "
                    "(seeds 440-%d), tol 1e-8, A = D_hat^+ D_hat; EigCG nev 10, m 60, max 300 vectors, "
                    "collecting on the first %d" % (args.eig_eps, kappa, mu, nrhs, 439 + nrhs, ncol),
        "cg": {"total_ms": round(sum(cg_ms), 1), "iters": cg_it, "ms": [round(v, 1) for v in cg_ms]},
        "eigcg": {"total_ms": round(sum(eig_ms), 1), "iters": eig_it, "ms": [round(v, 1) for v in eig_ms],
                  "max_true_rel_resid": max(eig_res), "lowest_ritz": [round(r, 8) for r in sorted(ritz)[:5]]},
        "eigcg_loop_no_deflation": {"ms": round(plain_loop_ms, 1), "iters": info0["iters"]},
        "speedup_total": round(sum(cg_ms) / sum(eig_ms), 3),
        "speedup_deflated_rhs": (round(sum(cg_ms[tail]) / sum(eig_ms[tail]), 3) if nrhs > ncol else None),
        "iteration_ratio_last": round(cg_it[-1] / max(1, eig_it[-1]), 3)}))
    lat.close()


def run_access(args):
    """The paper's addressing experiment on the isolated link-spinor kernel
    psi(x_i) = U(x_i) phi(x_i) (FP64; 144 B of link + 192 B in + 192 B out per site):
    sequential sites, sites through a random permutation index, and the same random
    sites through precomputed address arrays, in the site-major layout and in blocks
    of 64 sites, from 2^12 sites (cache-resident) to 2^24 (9 GB, HBM-bound)."""
    import torch
    from paper_1405_0700_amd import wilson as W
    gen = torch.Generator(device="cuda")
    gen.manual_seed(730)
    rows = []
    for lg in (12, 14, 16, 18, 20, 22, 24):
        n = 1 << lg
        u = torch.randn(n * 18, dtype=torch.float64, device="cuda", generator=gen)
        phi = torch.randn(n * 24, dtype=torch.float64, device="cuda", generator=gen)
        psi = torch.zeros(n * 24, dtype=torch.float64, device="cuda")
        perm = torch.randperm(n, device="cuda", generator=gen)
        idx = perm.to(torch.int32)
        for layout in (0, 1):
            def off(nc):
                if layout == 0:
                    return perm * (nc * 16)
                return ((perm // 64) * 64 * nc + perm % 64) * 16
            ptrs = torch.stack([psi.data_ptr() + off(12), u.data_ptr() + off(9), phi.data_ptr() + off(12)], 1)
            ptrs = ptrs.reshape(-1).contiguous()
            for mode, name, extra in ((W.WL_ACCESS_SEQ, "sequential", 0), (W.WL_ACCESS_INDEX, "index", 4),
                                      (W.WL_ACCESS_PTR, "pointers", 24)):
                call = lambda: W.wl_su3_apply(psi, u, phi, n, mode, layout, idx, ptrs)
                for _ in range(3):
                    call()
                reps = max(5, min(2000, (40 << 20) // n))
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(reps):
                    call()
                e1.record()
                torch.cuda.synchronize()
                us = e0.elapsed_time(e1) / reps * 1e3
                rows.append({"sites": n, "layout": "site-major" if layout == 0 else "64-site blocks", "mode": name,
                             "us": round(us, 2), "GBps": round(528 * n / us / 1e3, 1),
                             "GBps_with_addressing": round((528 + extra) * n / us / 1e3, 1)})
                print("[bench] %s" % rows[-1], file=sys.stderr, flush=True)
            del ptrs
        del u, phi, psi, perm, idx
        torch.cuda.empty_cache()
    print(json.dumps({"metric": "link-spinor kernel GB/s by addressing scheme and size", "unit": "GB/s",
                      "higher_is_better": True, "bytes_per_site": 528, "peak_GBps": HBM_PEAK_GBS,
                      "workload": "psi(x_i) = U(x_i) phi(x_i), FP64, torch.randn fields and permutation "
                                  "(generator seed 730), 2^12 .. 2^24 sites",
                      "results": rows}))


def run_split(args):
    """Half-dslash H_eo in on 24^3x48 and 32^3x64 (links exp(0.2iH) seeds 740/741, Gaussian
    input): the fused kernel (default launch, and one thread per point), and the bulk /
    boundary split form (t-face pack, face transfer on a second stream, bulk, boundary)
    that a rank of a t-decomposed lattice would run.  Algorithmic bytes per output site:
    8 links + input + output spinor."""
    import torch
    from paper_1405_0700_amd import synth
    from paper_1405_0700_amd import wilson as W
    rows = []
    for dims, seed in (((24, 24, 24, 48), 740), ((32, 32, 32, 64), 741)):
        lat = W.Lattice.create(synth.su3_links(dims, 0.2, seed), (1, 1, 1, -1))
        vh = lat.volume // 2
        src = synth.gaussian_spinor(dims, seed=seed + 100, nsites=vh)
        default = {p: W.wl_ctx_get_launch(lat.ctx, p) for p in (W.WL_F64, W.WL_F32)}
        for prec, recon, link_b, sp_b in ((W.WL_F64, 18, 144, 192), (W.WL_F32, 18, 72, 96), (W.WL_F32, 12, 48, 96)):
            inp = lat.pack(src, W.WL_ODD, prec)
            out = lat.new(W.WL_EVEN, prec)
            calls = {
                "fused": lambda: W.wl_dslash_apply(lat.ctx, out, inp, W.WL_EVEN, prec, recon),
                "split": lambda: W.wl_dslash_apply_split(lat.ctx, out, inp, W.WL_EVEN, prec, recon),
            }
            res = {}
            for name, tps in (("fused", None), ("fused_tps1", 1), ("split", None)):
                if tps:
                    W.wl_ctx_set_launch(lat.ctx, prec, 256, 1, tps)
                else:
                    W.wl_ctx_set_launch(lat.ctx, prec, *default[prec])
                fn = calls["split" if name == "split" else "fused"]
                for _ in range(5):
                    fn()
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(50):
                    fn()
                e1.record()
                torch.cuda.synchronize()
                us = e0.elapsed_time(e1) / 50 * 1e3
                res[name] = {"us": round(us, 2), "GBps": round((8 * link_b + 2 * sp_b) * vh / us / 1e3, 1)}
            W.wl_ctx_set_launch(lat.ctx, prec, *default[prec])
            rows.append({"dims": list(dims), "prec": {W.WL_F64: "f64", W.WL_F32: "f32"}[prec], "recon": recon,
                         "boundary_sites_fraction": round(2 / dims[3], 4), **res,
                         "split_over_fused": round(res["split"]["us"] / res["fused"]["us"], 3)})
            print("[bench] %s" % rows[-1], file=sys.stderr, flush=True)
        lat.close()
    print(json.dumps({"metric": "half-dslash time: bulk / boundary split with t-face transfer vs fused",
                      "unit": "us", "higher_is_better": False, "results": rows}))


if __name__ == "__main__":
    main()
