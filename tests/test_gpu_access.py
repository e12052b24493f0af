"""GPU parity of the link-spinor access kernel (wl_su3_apply) against the oracle:
psi(x_i) = U(x_i) phi(x_i) in the three addressing modes (sequential, index array,
precomputed addresses) and both layouts (site-major, blocks of 64 sites), at a ragged
size, plus argument errors and a sampled check at 2^22 sites.  FP64: the two sides sum
the three products of each row in different orders, so they agree to rounding
(1e-15 relative to the row's magnitude, which is that of phi for unitary U)."""

import numpy as np
import pytest
import torch

from oracle import oracle as orc
from paper_1405_0700_amd import synth
from paper_1405_0700_amd import wilson as W

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _announce(request):
    print("\n[gpu case] %s" % request.node.nodeid, flush=True)
    yield


def to_layout(a, layout):
    """(n, nc) complex site-major -> flat complex array of the layout (padded to 64 sites)."""
    n, nc = a.shape
    if layout == 0:
        return np.ascontiguousarray(a).ravel()
    nb = (n + 63) // 64
    pad = np.zeros((nb * 64, nc), dtype=np.complex128)
    pad[:n] = a
    return np.ascontiguousarray(pad.reshape(nb, 64, nc).transpose(0, 2, 1)).ravel()


def from_layout(flat, n, nc, layout):
    if layout == 0:
        return flat.reshape(-1, nc)[:n]
    nb = (n + 63) // 64
    return flat.reshape(nb, nc, 64).transpose(0, 2, 1).reshape(nb * 64, nc)[:n]


def site_offset(x, nc, layout):
    x = np.asarray(x, dtype=np.int64)
    if layout == 0:
        return x * nc * 16
    return ((x // 64) * 64 * nc + x % 64) * 16


def dev(a):
    return torch.from_numpy(a.view(np.float64).copy()).cuda()


def run(u, phi, psi0, mode, layout, sites):
    n = u.shape[0]
    du, dphi, dpsi = dev(to_layout(u.reshape(n, 9), layout)), dev(to_layout(phi.reshape(n, 12), layout)), \
        dev(to_layout(psi0.reshape(n, 12), layout))
    idx = ptrs = None
    if mode == W.WL_ACCESS_INDEX:
        idx = torch.from_numpy(np.asarray(sites, dtype=np.int32)).cuda()
    elif mode == W.WL_ACCESS_PTR:
        p = np.empty((len(sites), 3), dtype=np.uint64)
        p[:, 0] = dpsi.data_ptr() + site_offset(sites, 12, layout)
        p[:, 1] = du.data_ptr() + site_offset(sites, 9, layout)
        p[:, 2] = dphi.data_ptr() + site_offset(sites, 12, layout)
        ptrs = torch.from_numpy(p.view(np.int64).ravel().copy()).cuda()
    W.wl_su3_apply(dpsi, du, dphi, len(sites), mode, layout, idx, ptrs)
    torch.cuda.synchronize()
    out = dpsi.cpu().numpy().view(np.complex128)
    return from_layout(out, n, 12, layout).reshape(n, 4, 3)


def inputs(n, seed):
    rng = np.random.default_rng(seed)
    u = synth.haar_su3((n,), seed)
    phi = rng.standard_normal((n, 4, 3)) + 1j * rng.standard_normal((n, 4, 3))
    psi = rng.standard_normal((n, 4, 3)) + 1j * rng.standard_normal((n, 4, 3))
    return u, phi, psi


@pytest.mark.parametrize("layout", [0, 1])
@pytest.mark.parametrize("mode", [W.WL_ACCESS_SEQ, W.WL_ACCESS_INDEX, W.WL_ACCESS_PTR])
def test_matches_the_oracle(mode, layout):
    n = 3001  # several 256-thread blocks and a ragged 64-site block
    u, phi, psi = inputs(n, 700 + mode)
    sites = np.arange(n) if mode == W.WL_ACCESS_SEQ else np.random.default_rng(701).permutation(n)
    got = run(u, phi, psi, mode, layout, sites)
    ref = orc.su3_apply(u, phi, psi, sites)
    scale = np.abs(phi).max()
    assert np.max(np.abs(got - ref)) <= 1e-15 * 4 * scale


@pytest.mark.parametrize("mode", [W.WL_ACCESS_INDEX, W.WL_ACCESS_PTR])
def test_partial_and_repeated_sites(mode):
    """An index that visits some sites twice and others never: unvisited psi unchanged."""
    n = 700
    u, phi, psi = inputs(n, 710)
    sites = np.random.default_rng(711).integers(0, n, size=400)
    got = run(u, phi, psi, mode, 1, sites)
    ref = orc.su3_apply(u, phi, psi, sites)
    assert np.max(np.abs(got - ref)) <= 4e-15 * np.abs(phi).max()
    untouched = np.setdiff1d(np.arange(n), sites)
    assert np.array_equal(got[untouched], psi[untouched])


def test_large_sampled():
    """2^22 sites, blocks of 64, index mode over a permutation: 2000 sampled sites against the oracle."""
    n = 1 << 22
    rng = np.random.default_rng(720)
    u = synth.haar_su3((n,), 721)
    phi = rng.standard_normal((n, 4, 3)) + 1j * rng.standard_normal((n, 4, 3))
    psi = np.zeros((n, 4, 3), dtype=np.complex128)
    perm = rng.permutation(n)
    got = run(u, phi, psi, W.WL_ACCESS_INDEX, 1, perm)
    sample = rng.choice(n, 2000, replace=False)
    ref = orc.su3_apply(u[sample], phi[sample], psi[sample], range(len(sample)))
    assert np.max(np.abs(got[sample] - ref)) <= 4e-15 * np.abs(phi).max()


def test_argument_errors():
    x = torch.zeros(64 * 24, dtype=torch.float64, device="cuda")
    W.wl_su3_apply(x, x, x, 0)  # empty: nothing to do
    for kw in ({"mode": 3}, {"layout": 2}, {"mode": W.WL_ACCESS_INDEX}, {"mode": W.WL_ACCESS_PTR}):
        with pytest.raises(W.WilsonError):
            W.wl_su3_apply(x, x, x, 10, **kw)
    with pytest.raises(W.WilsonError):
        W.wl_su3_apply(x, x, x, -1)
    with pytest.raises(W.WilsonError):
        W.wl_su3_apply(None, x, x, 10)
