"""GPU tests of the bulk / boundary split hopping term (wl_dslash_apply_split), the paper's
scheme for overlapping communication with computation on a lattice decomposed in t: face
pack (the backward face multiplied by U_t^+ on the sending side), face transfer on a second
stream while the bulk computes, boundary completion.  It must equal the fused kernel with
one thread per point bit for bit (the same hops added in the same order), and the default
fused launch and the oracle to rounding, for both output parities, the adjoint, FP64 and
FP32 storage, 18 and 12 reals per link, random complex boundary phases, and the shortest
time extent (Lt = 2, where every site is on a boundary slice)."""

import numpy as np
import pytest
import torch

from oracle import oracle as orc
from paper_1405_0700_amd import synth
from paper_1405_0700_amd import wilson as W

pytestmark = pytest.mark.gpu
TOL = {W.WL_F64: 1e-13, W.WL_F32: 2e-6}


@pytest.fixture(autouse=True)
def _announce(request):
    print("\n[gpu case] %s" % request.node.nodeid, flush=True)
    yield


def rel(a, b):
    a, b = np.asarray(a).ravel(), np.asarray(b).ravel()
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("dims", [(8, 8, 8, 8), (6, 10, 4, 14), (4, 4, 4, 2), (16, 16, 16, 32)])
@pytest.mark.parametrize("prec,recon", [(W.WL_F64, 18), (W.WL_F64, 12), (W.WL_F32, 18), (W.WL_F32, 12)])
@pytest.mark.parametrize("dagger", [False, True])
def test_split_equals_fused(dims, prec, recon, dagger):
    rng = np.random.default_rng(31)
    ph = tuple(np.exp(1j * rng.uniform(0, 2 * np.pi, 4)))
    u = synth.su3_links(dims, 0.5, 32)
    lat = W.Lattice.create(u, ph)
    phi = synth.gaussian_spinor(dims, seed=33)
    want = orc.hop(phi, u, ph, dagger=dagger)
    we, wo = orc.eo_split(want, dims)
    pe, po = orc.eo_split(phi, dims)
    fused = W.wl_dslash_dagger_apply if dagger else W.wl_dslash_apply
    default_launch = W.wl_ctx_get_launch(lat.ctx, prec)
    for out_par, src, src_par, ref_half in ((W.WL_EVEN, po, W.WL_ODD, we), (W.WL_ODD, pe, W.WL_EVEN, wo)):
        inp = lat.pack(src, src_par, prec)
        got = lat.new(out_par, prec)
        W.wl_dslash_apply_split(lat.ctx, got, inp, out_par, prec, recon, dagger)
        one = lat.new(out_par, prec)
        W.wl_ctx_set_launch(lat.ctx, prec, 256, 1, 1)
        fused(lat.ctx, one, inp, out_par, prec, recon)
        dflt = lat.new(out_par, prec)
        W.wl_ctx_set_launch(lat.ctx, prec, *default_launch)
        fused(lat.ctx, dflt, inp, out_par, prec, recon)
        torch.cuda.synchronize()
        g = lat.unpack(got, out_par, prec)
        assert rel(g, ref_half) < TOL[prec]
        assert rel(g, lat.unpack(dflt, out_par, prec)) < TOL[prec]
        if not torch.equal(got, one):
            o = lat.unpack(one, out_par, prec).reshape(-1, 12)
            d = np.abs(g.reshape(-1, 12) - o).max(axis=1)
            bad = np.nonzero(d)[0]
            st = dims[0] * dims[1] * dims[2] // 2
            print("differing sites", len(bad), "of", len(d), "max", d.max(), "rel", d.max() / np.abs(o).max(),
                  "t slices", sorted(set((bad // st).tolist()))[:10])
        assert torch.equal(got, one)
    lat.close()


def test_split_repeated_calls_and_streams():
    """Back-to-back calls reuse the face buffers: each must see its own input."""
    dims = (8, 8, 8, 16)
    u = synth.su3_links(dims, 0.3, 34)
    lat = W.Lattice.create(u, (1, 1, 1, -1))
    fields = [synth.gaussian_spinor(dims, seed=35 + k, nsites=synth.volume(dims) // 2) for k in range(3)]
    ins = [lat.pack(f, W.WL_ODD) for f in fields]
    outs = [lat.new(W.WL_EVEN) for _ in fields]
    for i, o in zip(ins, outs):
        W.wl_dslash_apply_split(lat.ctx, o, i, W.WL_EVEN)
    W.wl_ctx_set_launch(lat.ctx, W.WL_F64, 256, 1, 1)
    for i, o in zip(ins, outs):
        ref = lat.new(W.WL_EVEN)
        W.wl_dslash_apply(lat.ctx, ref, i, W.WL_EVEN, W.WL_F64, 18)
        torch.cuda.synchronize()
        assert torch.equal(o, ref)
    lat.close()


def test_split_rejects_unsupported():
    dims = (4, 4, 4, 4)
    lat = W.Lattice.create(synth.su3_links(dims, 0.3, 36), (1, 1, 1, -1))
    with pytest.raises(W.WilsonError):
        W.wl_dslash_apply_split(lat.ctx, lat.new(W.WL_FULL), lat.new(W.WL_FULL), W.WL_FULL)
    with pytest.raises(W.WilsonError):
        W.wl_dslash_apply_split(lat.ctx, lat.new(W.WL_EVEN, W.WL_F16N), lat.new(W.WL_ODD, W.WL_F16N), W.WL_EVEN,
                                W.WL_F16N, 12)
    x = lat.new(W.WL_EVEN)
    with pytest.raises(W.WilsonError):
        W.wl_dslash_apply_split(lat.ctx, x, x, W.WL_EVEN)
    lat.close()
