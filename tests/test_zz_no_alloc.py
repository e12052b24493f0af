"""The allocation-free dot product (wl_blas_dot_noalloc) against wl_blas_dot, through the C ABI.

Two calls in a row, the second on a smaller input, so that what the first call left in the shared
static scratch array cannot leak into the second; both compared bit for bit with wl_blas_dot (the
same kernels and summation order).  An input whose partial sums exceed the array is rejected with
WL_ERR_ARG before anything is launched.
"""

import numpy as np
import pytest
import torch

from paper_1405_0700_amd import synth
from paper_1405_0700_amd import wilson as W

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _announce(request):
    print("\n[gpu case] %s" % request.node.nodeid, flush=True)
    yield


def _fields(lat, dims, subset, prec, nrhs, seed):
    nsite = lat.volume if subset == W.WL_FULL else lat.volume // 2
    xs = np.stack([synth.gaussian_spinor(dims, seed=seed + r, nsites=nsite) for r in range(nrhs)])
    ys = np.stack([synth.gaussian_spinor(dims, seed=seed + 50 + r, nsites=nsite) for r in range(nrhs)])
    return lat.pack(xs, subset, prec, nrhs), lat.pack(ys, subset, prec, nrhs)


def test_noalloc_dot_equals_dot_on_two_calls():
    cases = [((8, 8, 8, 16), W.WL_FULL, W.WL_F64, 3, 11), ((4, 4, 4, 8), W.WL_EVEN, W.WL_F32, 1, 12)]
    for dims, subset, prec, nrhs, seed in cases:
        lat = W.Lattice.create(synth.su3_links(dims, 0.3, seed), (1, 1, 1, -1))
        try:
            x, y = _fields(lat, dims, subset, prec, nrhs, seed)
            res = torch.full((2,), float("nan"), dtype=torch.float64, device="cuda")
            W.wl_blas_dot_noalloc(lat.ctx, x, y, subset, prec, nrhs, res)
            torch.cuda.synchronize()
            got = res.cpu().numpy()
            want = W.wl_blas_dot(lat.ctx, x, y, subset, prec, nrhs)
            print(dims, subset, prec, nrhs, got, want)
            assert got[0] == want.real and got[1] == want.imag
        finally:
            lat.close()


def test_noalloc_dot_rejects_inputs_beyond_its_scratch():
    dims = (32, 32, 32, 8)
    lat = W.Lattice.create(synth.su3_links(dims, 0.1, 13), (1, 1, 1, -1))
    try:
        small = torch.zeros(1024, dtype=torch.uint8, device="cuda")
        res = torch.zeros(2, dtype=torch.float64, device="cuda")
        with pytest.raises(W.WilsonError) as ei:
            W.wl_blas_dot_noalloc(lat.ctx, small, small, W.WL_FULL, W.WL_F64, 64, res)
        assert ei.value.status == W.WL_ERR_ARG and "scratch" in str(ei.value)
        torch.cuda.synchronize()
        assert not torch.any(res)
    finally:
        lat.close()
