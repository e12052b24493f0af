"""Kernel timing through the C-ABI: every n-th hopping launch is recorded, per kernel kind."""

import pytest
import torch

from paper_1405_0700_amd import synth
from paper_1405_0700_amd import wilson as W

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _announce(request):
    print("\n[gpu case] %s" % request.node.nodeid, flush=True)
    yield


def test_timing_records_every_nth_launch():
    dims = (8, 8, 8, 8)
    lat = W.Lattice.create(synth.su3_links(dims, 0.3, 60), (1, 1, 1, -1))
    inp = lat.pack(synth.gaussian_spinor(dims, seed=61, nsites=lat.volume // 2), W.WL_ODD)
    out = lat.new(W.WL_EVEN)
    for every, want in ((1, 7), (3, 3)):
        W.wl_timing_enable(lat.ctx, True, every=every)
        for _ in range(7):
            W.wl_dslash_apply(lat.ctx, out, inp, W.WL_EVEN, W.WL_F64, 18)
        torch.cuda.synchronize()
        n, ms = W.wl_timing_read(lat.ctx, W.WL_F64, 18, False, 0)
        assert n == want and ms > 0.0
        n_dag, _ = W.wl_timing_read(lat.ctx, W.WL_F64, 18, True, 0)
        assert n_dag == 0
    W.wl_timing_enable(lat.ctx, False)
    W.wl_dslash_apply(lat.ctx, out, inp, W.WL_EVEN, W.WL_F64, 18)
    assert W.wl_timing_read(lat.ctx, W.WL_F64, 18, False, 0)[0] == 0
    with pytest.raises(W.WilsonError):
        W.wl_timing_enable(lat.ctx, True, every=-1)
    lat.close()
