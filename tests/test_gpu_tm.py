"""GPU parity of the twisted-mass operator (D_tm = 1 + 2 i kappa mu gamma_5 - kappa H
and its even/odd Schur complement) and of CG with a twisted mass, against the FP64
oracle, through the C ABI.  Tolerances as for the Wilson operator (storage-format
dependent); solves are judged by the oracle-restated residual."""

import numpy as np
import pytest
import torch

from oracle import oracle as orc
from paper_1405_0700_amd import synth
from paper_1405_0700_amd import wilson as W

pytestmark = pytest.mark.gpu
TOL = {W.WL_F64: 1e-13, W.WL_F32: 2e-6, W.WL_F16N: 4e-3}
AP = (1, 1, 1, -1)


@pytest.fixture(autouse=True)
def _announce(request):
    print("\n[gpu case] %s" % request.node.nodeid, flush=True)
    yield


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def random_phases(seed):
    rng = np.random.default_rng(seed)
    return tuple(np.exp(1j * rng.uniform(0, 2 * np.pi, 4)))


def rounded(f, prec):
    return f.astype(np.complex64).astype(np.complex128) if prec != W.WL_F64 else f


DIMS = (6, 4, 4, 8)


@pytest.mark.parametrize("prec,recon", [(W.WL_F64, 18), (W.WL_F32, 12), (W.WL_F16N, 12)])
@pytest.mark.parametrize("dagger", [False, True])
@pytest.mark.parametrize("tps", [1, 2])
def test_twisted_operators_match_oracle(prec, recon, dagger, tps):
    ph = random_phases(820)
    u = synth.su3_links(DIMS, 0.5, 821)
    lat = W.Lattice.create(u, ph)
    if prec != W.WL_F16N:
        W.wl_ctx_set_launch(lat.ctx, prec, 128, 1, tps, 0, -1)
    kappa, mu = 0.125, 0.31
    phi = synth.gaussian_spinor(DIMS, seed=822)
    inp = lat.pack(phi, W.WL_FULL, prec)
    phi_s = lat.unpack(inp, W.WL_FULL, prec).reshape(phi.shape)  # the stored (rounded) input
    out = lat.new(W.WL_FULL, prec)
    W.wl_dirac_tm_apply(lat.ctx, out, inp, W.WL_OP_D, dagger, kappa, mu, prec, recon)
    want = orc.dirac_tm(phi_s, u, kappa, mu, ph, dagger)
    assert rel(lat.unpack(out, W.WL_FULL, prec).reshape(want.shape), want) < TOL[prec]
    pe, _ = orc.eo_split(phi, DIMS)
    ine = lat.pack(pe, W.WL_EVEN, prec)
    pe_s = lat.unpack(ine, W.WL_EVEN, prec)
    oe = lat.new(W.WL_EVEN, prec)
    W.wl_dirac_tm_apply(lat.ctx, oe, ine, W.WL_OP_DHAT, dagger, kappa, mu, prec, recon)
    want = orc.schur_tm(pe_s, u, kappa, mu, ph, dagger)
    assert rel(lat.unpack(oe, W.WL_EVEN, prec), want) < TOL[prec]
    lat.close()


def test_mu_zero_is_bitwise_wilson():
    ph = random_phases(823)
    u = synth.su3_links(DIMS, 0.5, 824)
    lat = W.Lattice.create(u, ph)
    inp = lat.pack(synth.gaussian_spinor(DIMS, seed=825))
    a, b = lat.new(W.WL_FULL), lat.new(W.WL_FULL)
    W.wl_dirac_apply(lat.ctx, a, inp, W.WL_OP_D, False, 0.13)
    W.wl_dirac_tm_apply(lat.ctx, b, inp, W.WL_OP_D, False, 0.13, 0.0)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    lat.close()


def test_twisted_even_odd_helpers():
    ph = random_phases(826)
    u = synth.su3_links(DIMS, 0.5, 827)
    lat = W.Lattice.create(u, ph)
    kappa, mu = 0.12, 0.4
    b = synth.gaussian_spinor(DIMS, seed=828)
    x = synth.gaussian_spinor(DIMS, seed=829)
    be, bo = orc.eo_split(b, DIMS)
    xe, _ = orc.eo_split(x, DIMS)
    bh = lat.new(W.WL_EVEN)
    W.wl_eo_prepare_tm(lat.ctx, bh, lat.pack(be, W.WL_EVEN), lat.pack(bo, W.WL_ODD), kappa, mu)
    assert rel(lat.unpack(bh, W.WL_EVEN), orc.eo_prepare_tm(be, bo, u, kappa, mu, ph)) < 1e-13
    xo = lat.new(W.WL_ODD)
    W.wl_eo_reconstruct_tm(lat.ctx, xo, lat.pack(xe, W.WL_EVEN), lat.pack(bo, W.WL_ODD), kappa, mu)
    assert rel(lat.unpack(xo, W.WL_ODD), orc.eo_reconstruct_tm(xe, bo, u, kappa, mu, ph)) < 1e-13
    lat.close()


@pytest.mark.parametrize("prec,recon", [(W.WL_F64, 18), (W.WL_F32, 18), (W.WL_F16N, 12)])
def test_twisted_mass_even_odd_solve(prec, recon):
    """Full solve of D_tm x = eta through the Schur complement: prepare, D_hat_tm^+ of the
    source, CG on the normal equations (FP64 or mixed with FP64 reliable updates),
    reconstruct; judged by the oracle's ||eta - D_tm x|| / ||eta||."""
    dims = (8, 8, 8, 8)
    ph = AP
    u = synth.su3_links(dims, 0.3, 830)
    lat = W.Lattice.create(u, ph)
    kappa, mu = 0.13, 0.05
    eta = synth.gaussian_spinor(dims, seed=831)
    be, bo = orc.eo_split(eta, dims)
    Be, Bo = lat.pack(be, W.WL_EVEN), lat.pack(bo, W.WL_ODD)
    bhat = lat.new(W.WL_EVEN)
    W.wl_eo_prepare_tm(lat.ctx, bhat, Be, Bo, kappa, mu)
    rhs = lat.new(W.WL_EVEN)
    W.wl_dirac_tm_apply(lat.ctx, rhs, bhat, W.WL_OP_DHAT, True, kappa, mu)
    p = W.wl_solver_params_default()
    p.prec, p.recon, p.mu, p.tol = prec, recon, mu, 1e-11
    xe = lat.new(W.WL_EVEN)
    st, info = W.wl_cg_solve(lat.ctx, xe, rhs, W.WL_OP_DHAT, kappa, params=p)
    assert st == W.WL_OK
    xo = lat.new(W.WL_ODD)
    W.wl_eo_reconstruct_tm(lat.ctx, xo, xe, Bo, kappa, mu)
    x = orc.eo_join(lat.unpack(xe, W.WL_EVEN), lat.unpack(xo, W.WL_ODD), dims)
    r = rel(orc.dirac_tm(x, u, kappa, mu, ph), eta)
    print("prec", prec, info[0], "oracle residual", r)
    assert r < 1e-9
    lat.close()


def test_twisted_mass_batch_solve_matches_single():
    ph = AP
    systems = [((4, 4, 4, 8), 840), ((6, 4, 4, 4), 841)]
    lats, rhs, gauges = [], [], []
    kappa, mu = 0.12, 0.2
    for dims, seed in systems:
        u = synth.su3_links(dims, 0.4, seed)
        lat = W.Lattice.create(u, ph)
        lats.append(lat)
        gauges.append(u)
        rhs.append(lat.pack(synth.gaussian_spinor(dims, seed=seed + 1, nsites=synth.volume(dims) // 2), W.WL_EVEN))
    b = W.wl_batch_create([l.ctx for l in lats])
    p = W.wl_solver_params_default()
    p.mu, p.tol = mu, 1e-10
    xs = [l.new(W.WL_EVEN) for l in lats]
    st, info = W.wl_batch_cg_solve(b, xs, rhs, W.WL_OP_DHAT, [kappa, kappa], 1, p)
    assert st == W.WL_OK
    for k, ((dims, _), lat, u) in enumerate(zip(systems, lats, gauges)):
        x = lat.unpack(xs[k], W.WL_EVEN)
        a = orc.schur_tm(orc.schur_tm(x, u, kappa, mu, ph), u, kappa, mu, ph, dagger=True)
        assert rel(a, lat.unpack(rhs[k], W.WL_EVEN)) <= 1.05e-10
    W.wl_batch_destroy(b)
