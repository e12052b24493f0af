"""GPU parity of the batch path: one persistent launch of the hopping term over
several lattices of different sizes (each with its own gauge field, kappa and
right-hand sides), and CG on all of them in lockstep.

Every output point of the persistent kernel is computed by the same per-point
code as the one-thread-per-point kernel of a single context, so the batch
operator equals the single-context operator (tps = 1) bit for bit, whatever the
tile size and number of workgroups (with the same threads per point); against the oracle it holds the per-op
bar of 1e-13 (FP64) / the storage tolerances (FP32).  Batched solves are
judged by the oracle-restated residual of every system and right-hand side.
"""

import numpy as np
import pytest
import torch

from oracle import oracle as orc
from paper_1405_0700_amd import synth
from paper_1405_0700_amd import wilson as W

pytestmark = pytest.mark.gpu
AP = (1, 1, 1, -1)
SYSTEMS = [((4, 4, 4, 4), 0.5, 701, 0.12), ((6, 6, 4, 8), 0.5, 702, 0.11), ((8, 4, 6, 4), 0.4, 703, 0.125)]


@pytest.fixture(autouse=True)
def _announce(request):
    print("\n[gpu case] %s" % request.node.nodeid, flush=True)
    yield


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


@pytest.fixture(scope="module")
def batch():
    lats, gauges = [], []
    for dims, eps, seed, _ in SYSTEMS:
        u = synth.su3_links(dims, eps, seed)
        lats.append(W.Lattice.create(u, AP))
        gauges.append(u)
    b = W.wl_batch_create([l.ctx for l in lats])
    yield b, lats, gauges
    W.wl_batch_destroy(b)


def stacked(dims, seeds):
    return np.stack([synth.gaussian_spinor(dims, seed=s).reshape(-1, 4, 3) for s in seeds])


@pytest.mark.parametrize("op", [W.WL_OP_D, W.WL_OP_DHAT])
@pytest.mark.parametrize("dagger", [False, True])
@pytest.mark.parametrize("nrhs", [1, 4])
@pytest.mark.parametrize("tps", [1, 2])
def test_batch_operator_matches_single_context_and_oracle(batch, op, dagger, nrhs, tps):
    b, lats, gauges = batch
    saved = W.wl_batch_get_launch(b)
    W.wl_batch_set_launch(b, saved[0], 256, -1, tps)
    subset = W.WL_FULL if op == W.WL_OP_D else W.WL_EVEN
    kappas = [s[3] for s in SYSTEMS]
    ins, outs, fields = [], [], []
    for k, (lat, (dims, _, seed, _)) in enumerate(zip(lats, SYSTEMS)):
        f = stacked(dims, [seed * 10 + r for r in range(nrhs)])
        if subset == W.WL_EVEN:
            f = np.stack([orc.eo_split(g.reshape(dims[::-1] + (4, 3)), dims)[0] for g in f])
        fields.append(f)
        ins.append(lat.pack(f if nrhs > 1 else f[0], subset, W.WL_F64, nrhs))
        outs.append(lat.new(subset, W.WL_F64, nrhs))
    W.wl_batch_dirac_apply(b, outs, ins, op, dagger, kappas, W.WL_F64, 18, nrhs)
    W.wl_batch_set_launch(b, *saved)
    for k, (lat, u, (dims, _, _, kappa)) in enumerate(zip(lats, gauges, SYSTEMS)):
        # single context with the same threads per point: the same per-point code
        W.wl_ctx_set_launch(lat.ctx, W.WL_F64, 256, 1, tps, 0, -1)
        ref = lat.new(subset, W.WL_F64, nrhs)
        W.wl_dirac_apply(lat.ctx, ref, ins[k], op, dagger, kappa, W.WL_F64, 18, nrhs)
        torch.cuda.synchronize()
        assert torch.equal(outs[k], ref), "system %d" % k
        W.wl_ctx_set_launch(lat.ctx, W.WL_F64, 128, 1, 2, 0, -1)
        got = lat.unpack(outs[k], subset, W.WL_F64, nrhs)
        got = got if nrhs > 1 else got[None]
        for r in range(nrhs):
            if op == W.WL_OP_D:
                want = orc.dirac(fields[k][r].reshape(dims[::-1] + (4, 3)), u, kappa, AP, dagger=dagger)
                assert rel(got[r].reshape(want.shape), want) < 1e-13
            else:
                want = orc.schur(fields[k][r], u, kappa, AP, dagger=dagger)
                assert rel(got[r], want) < 1e-13


@pytest.mark.parametrize("op", [W.WL_OP_D, W.WL_OP_DHAT])
@pytest.mark.parametrize("nrhs", [1, 3])
def test_batch_per_system_launches_equal_the_single_context_operator(batch, op, nrhs):
    # workgroups 0: each system is applied by its own context's launches, bit for bit
    b, lats, gauges = batch
    saved = W.wl_batch_get_launch(b)
    W.wl_batch_set_launch(b, 0, saved[1], saved[2], saved[3])
    assert W.wl_batch_get_launch(b)[0] == 0
    subset = W.WL_FULL if op == W.WL_OP_D else W.WL_EVEN
    kappas = [s[3] for s in SYSTEMS]
    ins, outs = [], []
    for lat, (dims, _, seed, _) in zip(lats, SYSTEMS):
        n = synth.volume(dims) // (1 if subset == W.WL_FULL else 2)
        f = np.stack([synth.gaussian_spinor(dims, seed=seed * 13 + r, nsites=n) for r in range(nrhs)])
        ins.append(lat.pack(f if nrhs > 1 else f[0], subset, W.WL_F64, nrhs))
        outs.append(lat.new(subset, W.WL_F64, nrhs))
    try:
        for dagger in (False, True):
            W.wl_batch_dirac_apply(b, outs, ins, op, dagger, kappas, W.WL_F64, 18, nrhs)
            for k, lat in enumerate(lats):
                ref = lat.new(subset, W.WL_F64, nrhs)
                W.wl_dirac_apply(lat.ctx, ref, ins[k], op, dagger, kappas[k], W.WL_F64, 18, nrhs)
                torch.cuda.synchronize()
                assert torch.equal(outs[k], ref), (k, dagger)
    finally:
        W.wl_batch_set_launch(b, *saved)


def test_batch_launch_shape_does_not_change_results_and_launches_repeat(batch):
    b, lats, _ = batch
    kappas = [s[3] for s in SYSTEMS]
    ins = [lat.pack(stacked(dims, [seed, seed + 1]), W.WL_FULL, W.WL_F32, 2)
           for lat, (dims, _, seed, _) in zip(lats, SYSTEMS)]
    default = W.wl_batch_get_launch(b)
    results = []
    # one workgroup per XCD, fewer workgroups than tiles, and many more workgroups than tiles
    for wg, blk in ((default[0], 256), (8, 64), (64, 128), (16, 256), (4096, 64), (default[0], 256)):
        W.wl_batch_set_launch(b, wg, blk, -1, default[3])
        outs = [lat.new(W.WL_FULL, W.WL_F32, 2) for lat in lats]
        # three launches in a row give the same result (no state carried between launches)
        for _ in range(3):
            W.wl_batch_dirac_apply(b, outs, ins, W.WL_OP_D, False, kappas, W.WL_F32, 18, 2)
        torch.cuda.synchronize()
        results.append([o.clone() for o in outs])
    W.wl_batch_set_launch(b, *default)
    for res in results[1:]:
        for k in range(len(lats)):
            assert torch.equal(res[k], results[0][k])


@pytest.mark.parametrize("prec,recon,use_graph,nt,tps", [
    (W.WL_F32, 18, 0, -1, 1), (W.WL_F32, 18, 1, -1, 1), (W.WL_F64, 18, 1, -1, 1), (W.WL_F64, 12, 0, -1, 1),
    (W.WL_F16N, 12, 1, -1, 1), (W.WL_BF16N, 12, 0, -1, 1),
    # non-temporal stores and two threads per point, as chosen for large lattices
    (W.WL_F32, 18, 1, 1, 2), (W.WL_F64, 18, 0, 1, 2), (W.WL_F16N, 12, 0, 1, 1),
    # nt = None: one launch per system (workgroups 0) with the contexts' own shapes
    (W.WL_F32, 18, 1, None, 1), (W.WL_F16N, 12, 0, None, 1), (W.WL_F64, 18, 0, None, 1)])
def test_batch_cg_mixed_precision_solves_every_system(batch, prec, recon, use_graph, nt, tps):
    b, lats, gauges = batch
    saved = W.wl_batch_get_launch(b)
    if nt is None:
        W.wl_batch_set_launch(b, 0, saved[1], saved[2], saved[3])
    else:
        W.wl_batch_set_launch(b, saved[0], saved[1], nt, tps)
    try:
        _batch_cg_case(b, lats, gauges, prec, recon, use_graph)
    finally:
        W.wl_batch_set_launch(b, *saved)


def _batch_cg_case(b, lats, gauges, prec, recon, use_graph):
    nrhs = 4
    kappas = [s[3] for s in SYSTEMS]
    xs, rhs, bhats = [], [], []
    for lat, u, (dims, _, seed, kappa) in zip(lats, gauges, SYSTEMS):
        etas = stacked(dims, [seed * 7 + r for r in range(nrhs)])
        be = np.stack([orc.eo_split(e.reshape(dims[::-1] + (4, 3)), dims)[0] for e in etas])
        bo = np.stack([orc.eo_split(e.reshape(dims[::-1] + (4, 3)), dims)[1] for e in etas])
        bhat = np.stack([orc.eo_prepare(be[r], bo[r], u, kappa, AP) for r in range(nrhs)])
        rhs_c = np.stack([orc.schur(bhat[r], u, kappa, AP, dagger=True) for r in range(nrhs)])
        bhats.append(rhs_c)
        rhs.append(lat.pack(rhs_c, W.WL_EVEN, W.WL_F64, nrhs))
        xs.append(lat.new(W.WL_EVEN, W.WL_F64, nrhs))
    p = W.wl_solver_params_default()
    p.prec, p.recon, p.use_graph, p.tol = prec, recon, use_graph, 1e-10
    st, info = W.wl_batch_cg_solve(b, xs, rhs, W.WL_OP_DHAT, kappas, nrhs, p)
    assert st == W.WL_OK
    for k, (lat, u, (dims, _, _, kappa)) in enumerate(zip(lats, gauges, SYSTEMS)):
        x = lat.unpack(xs[k], W.WL_EVEN, W.WL_F64, nrhs)
        for r in range(nrhs):
            a = orc.schur(orc.schur(x[r], u, kappa, AP), u, kappa, AP, dagger=True)
            assert rel(a, bhats[k][r]) <= 1.05e-10, (k, r)
            assert info[k][r]["true_rel_resid"] <= 1e-10 and info[k][r]["iters"] > 0
    print("iterations per system:", [[i["iters"] for i in s] for s in info])


@pytest.mark.parametrize("prec", [W.WL_F64, W.WL_F32])
def test_batch_cg_full_operator_solves_every_system(batch, prec):
    # M = D on the whole lattice: the fused residual update covers both parities
    b, lats, gauges = batch
    nrhs = 2
    kappas = [s[3] for s in SYSTEMS]
    xs, rhs, want = [], [], []
    for lat, u, (dims, _, seed, kappa) in zip(lats, gauges, SYSTEMS):
        etas = [synth.gaussian_spinor(dims, seed=seed * 11 + r) for r in range(nrhs)]
        rhs_c = np.stack([orc.dirac(e, u, kappa, AP, dagger=True).reshape(-1, 4, 3) for e in etas])
        want.append(rhs_c)
        rhs.append(lat.pack(rhs_c, W.WL_FULL, W.WL_F64, nrhs))
        xs.append(lat.new(W.WL_FULL, W.WL_F64, nrhs))
    p = W.wl_solver_params_default()
    p.prec, p.tol = prec, 1e-10
    st, info = W.wl_batch_cg_solve(b, xs, rhs, W.WL_OP_D, kappas, nrhs, p)
    assert st == W.WL_OK
    for k, (lat, u, (dims, _, _, kappa)) in enumerate(zip(lats, gauges, SYSTEMS)):
        x = lat.unpack(xs[k], W.WL_FULL, W.WL_F64, nrhs)
        for r in range(nrhs):
            xr = x[r].reshape(dims[::-1] + (4, 3))
            a = orc.dirac(orc.dirac(xr, u, kappa, AP), u, kappa, AP, dagger=True)
            assert rel(a.reshape(-1, 4, 3), want[k][r]) <= 1.05e-10, (k, r)
            assert info[k][r]["true_rel_resid"] <= 1e-10 and info[k][r]["iters"] > 0
    print("iterations per system:", [[i["iters"] for i in s] for s in info])


def test_batch_cg_graph_replay_equals_eager(batch):
    b, lats, gauges = batch
    kappas = [s[3] for s in SYSTEMS]
    rhs = [lat.pack(synth.gaussian_spinor(dims, seed=seed + 5, nsites=synth.volume(dims) // 2), W.WL_EVEN)
           for lat, (dims, _, seed, _) in zip(lats, SYSTEMS)]
    sols = []
    for g in (0, 1):
        xs = [lat.new(W.WL_EVEN) for lat in lats]
        p = W.wl_solver_params_default()
        p.prec, p.use_graph, p.tol, p.maxiter, p.max_restarts = W.WL_F32, g, 0.0, 60, 0
        p.reliable_every = 25
        W.wl_batch_cg_solve(b, xs, rhs, W.WL_OP_DHAT, kappas, 1, p)
        torch.cuda.synchronize()
        sols.append(xs)
    for k in range(len(lats)):
        assert torch.equal(sols[0][k], sols[1][k])


def test_batch_rejects_bad_arguments(batch):
    b, lats, _ = batch
    with pytest.raises(W.WilsonError):
        W.wl_batch_set_launch(b, 12, 256, -1)
    with pytest.raises(W.WilsonError):
        W.wl_batch_set_launch(b, 64, 96, -1)
    with pytest.raises(W.WilsonError):
        W.wl_batch_set_launch(b, 64, 256, -1, 3)
    with pytest.raises(W.WilsonError):
        W.wl_batch_create([lats[0].ctx, lats[0].ctx])
    outs = [lat.new(W.WL_FULL) for lat in lats]
    with pytest.raises(W.WilsonError):
        W.wl_batch_dirac_apply(b, outs, outs, W.WL_OP_D, False, [0.1, 0.1, 0.1])


# ------------------------------------------------------------------ autotuner
def test_autotune_picks_a_valid_launch_and_caches_it(tmp_path):
    dims = (8, 8, 8, 16)
    u = synth.su3_links(dims, 0.3, 711)
    lat = W.Lattice.create(u, AP)
    cache = tmp_path / "tune.txt"
    cfg, us, cached = W.wl_autotune(lat.ctx, W.WL_F32, 18, 1, cache)
    assert not cached and us > 0
    block, swizzle, tps, tchunk, nt, rpt, occ, sweep = cfg
    assert block in (64, 128, 256) and tps in (1, 2) and swizzle in (0, 1) and tchunk in (0, 4, W.WL_TCHUNK_AUTO, W.WL_TCHUNK_YZ) \
        and nt in (0, 1) and occ == 0 and sweep == 0
    assert rpt == 1  # one right-hand side: nothing to share
    assert W.wl_ctx_get_launch(lat.ctx, W.WL_F32) == cfg
    # the tuned launch still computes D (FP32 storage tolerance against the oracle)
    phi = synth.gaussian_spinor(dims, seed=712)
    out = lat.new(W.WL_FULL, W.WL_F32)
    W.wl_dirac_apply(lat.ctx, out, lat.pack(phi, W.WL_FULL, W.WL_F32), W.WL_OP_D, False, 0.12, W.WL_F32, 18)
    want = orc.dirac(phi.astype(np.complex64).astype(np.complex128), u, 0.12, AP)
    assert rel(lat.unpack(out, W.WL_FULL, W.WL_F32).reshape(want.shape), want) < 2e-6
    # in-process cache
    cfg2, us2, cached2 = W.wl_autotune(lat.ctx, W.WL_F32, 18, 1, cache)
    assert cached2 and cfg2 == cfg and us2 == pytest.approx(us, rel=1e-5)
    # file cache: an entry written by hand for another key is read back and applied
    line = cache.read_text().strip().splitlines()[-1]
    key = line.split(" | ")[0].replace("nrhs 1", "nrhs 3")
    with open(cache, "a") as f:
        f.write("garbage line without separator\n")
        f.write("%s | 64 0 1 0 0 3 12.5\n" % key)
    cfg3, us3, cached3 = W.wl_autotune(lat.ctx, W.WL_F32, 18, 3, cache)
    assert cached3 and cfg3 == (64, 0, 1, 0, 0, 3, 0, 0) and us3 == 12.5
    # an entry that is not a valid launch shape (block 1000) is ignored and the shape tuned again
    with open(cache, "a") as f:
        f.write("%s | 1000 0 1 0 0 1 1.0\n" % key.replace("nrhs 3", "nrhs 2"))
    cfg4, us4, cached4 = W.wl_autotune(lat.ctx, W.WL_F32, 18, 2, cache)
    assert not cached4 and cfg4[0] in (64, 128, 256) and us4 > 0
    assert W.wl_ctx_get_launch(lat.ctx, W.WL_F32) == cfg4
    lat.close()


def test_batch_autotune(batch, tmp_path):
    b, lats, _ = batch
    before = W.wl_batch_get_launch(b)
    (wg, blk, nt, tps), us, cached = W.wl_batch_autotune(b, W.WL_F32, 18, 2, tmp_path / "b.txt")
    # workgroups 0: one launch per system (then nt and tps are the batch's unused settings)
    assert not cached and us > 0 and wg % 8 == 0 and blk in (64, 128, 256) and nt in (-1, 0, 1) and tps in (1, 2)
    assert W.wl_batch_get_launch(b) == (wg, blk, nt, tps)
    again = W.wl_batch_autotune(b, W.WL_F32, 18, 2, tmp_path / "b.txt")
    assert again[2] and again[0] == (wg, blk, nt, tps)
    # an invalid cache entry (12 workgroups: not a multiple of 8) is ignored and the batch tuned again
    key = (tmp_path / "b.txt").read_text().strip().splitlines()[-1].split(" | ")[0].replace("nrhs 2", "nrhs 1")
    with open(tmp_path / "b.txt", "a") as f:
        f.write("%s | 12 256 0 1 1.0\n" % key)
    (wg5, blk5, nt5, tps5), us5, cached5 = W.wl_batch_autotune(b, W.WL_F32, 18, 1, tmp_path / "b.txt")
    assert not cached5 and wg5 % 8 == 0 and us5 > 0
    W.wl_batch_set_launch(b, *before)
