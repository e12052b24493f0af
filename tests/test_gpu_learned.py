"""The learned preconditioner end to end on small lattices, with the default
training recipe (pairs from the first iterations of plain CG, residual-norm
loss): harvested pairs satisfy r = D e, training with the library's own
forward/backward/Adam kernels lowers the loss, and FGCR and CG on the normal
equations of D M with the trained network need fewer iterations than without
a preconditioner and than with the untrained network, on a gauge field and
source it was not trained on."""

import numpy as np
import pytest

from oracle import oracle as orc
from oracle import ptc
from paper_1405_0700_amd import learned, synth
from paper_1405_0700_amd import wilson as W

pytestmark = pytest.mark.gpu
AP = (1, 1, 1, -1)
DIMS = (8, 8, 8, 8)
KAPPA = 0.137
# restarted FGCR with the untrained network stalls at kappa 0.137 on this field (with either network kernel):
# its comparison runs at 0.13
KAPPA_FGCR = 0.13


@pytest.fixture(autouse=True)
def _announce(request):
    print("\n[gpu case] %s" % request.node.nodeid, flush=True)
    yield


@pytest.fixture(scope="module")
def trained():
    sets, gauges = [], []
    for k in range(2):
        u = synth.su3_links(DIMS, 0.2, 600 + k)
        lat = W.Lattice.create(u, AP)
        srcs = [synth.gaussian_spinor(DIMS, seed=610 + 2 * k + j) for j in range(2)]
        sets.append((lat, learned.harvest(lat, srcs, KAPPA)))
        gauges.append(u)
    w1, w2 = synth.ptc_weights(8, seed=530)
    net = W.wl_ptc_create(w1, w2)
    losses = learned.train(sets, net, epochs=60, lr=1e-3, loss="residual", kappa=KAPPA)
    yield sets, gauges, net, losses
    W.wl_ptc_destroy(net)


def test_harvested_pairs_satisfy_r_equals_D_e(trained):
    sets, gauges, _, _ = trained
    lat, pairs = sets[0]
    r, e = pairs[1]
    rc = lat.unpack(r, W.WL_FULL, W.WL_F32).reshape(DIMS[::-1] + (4, 3))
    ec = lat.unpack(e, W.WL_FULL, W.WL_F32).reshape(DIMS[::-1] + (4, 3))
    de = orc.dirac(ec, gauges[0], KAPPA, AP)
    assert np.linalg.norm(de - rc) / np.linalg.norm(rc) < 1e-5


def test_training_lowers_the_loss(trained):
    _, _, _, losses = trained
    print("loss first %.5f last %.5f" % (losses[0], losses[-1]))
    assert np.all(np.isfinite(losses))
    assert losses[-1] < 0.8 * losses[0]


def test_fgcr_with_the_trained_network(trained):
    _, _, net, _ = trained
    u = synth.su3_links(DIMS, 0.2, 620)
    lat = W.Lattice.create(u, AP)
    b = synth.gaussian_spinor(DIMS, seed=621)
    res = {}
    fresh = W.wl_ptc_create(*synth.ptc_weights(8, seed=530))
    for name, m in (("none", None), ("initial", fresh), ("trained", net)):
        x = lat.new(W.WL_FULL)
        p = W.wl_fgcr_params_default()
        p.fallback = 0
        st, info = W.wl_fgcr_solve(lat.ctx, x, lat.pack(b), KAPPA_FGCR, m, p)
        xs = lat.unpack(x).reshape(b.shape)
        r = np.linalg.norm(orc.dirac(xs, u, KAPPA_FGCR, AP) - b) / np.linalg.norm(b)
        assert st == W.WL_OK and r <= 1.05e-10, (name, st, r)
        res[name] = info["iters"]
    print("FGCR iterations by preconditioner:", res)
    assert res["trained"] < res["initial"] and res["trained"] < res["none"]
    W.wl_ptc_destroy(fresh)
    lat.close()


def test_preconditioned_cgnr_with_the_trained_network(trained):
    _, _, net, _ = trained
    u = synth.su3_links(DIMS, 0.2, 620)
    lat = W.Lattice.create(u, AP)
    b = synth.gaussian_spinor(DIMS, seed=621)
    res = {}
    fresh = W.wl_ptc_create(*synth.ptc_weights(8, seed=530))
    # the first-order Neumann preconditioner M = 1 + kappa H as network weights: layer 1 passes the input to
    # channel 0, layer 2 applies the identity plus kappa (1 -/+ gamma_mu) along the forward / backward hops
    w1 = np.zeros((9, 8, 1, 4, 4), dtype=np.complex128)
    w2 = np.zeros((9, 1, 8, 4, 4), dtype=np.complex128)
    w1[0, 0, 0] = np.eye(4)
    w2[0, 0, 0] = np.eye(4)
    for mu in range(4):
        w2[1 + 2 * mu, 0, 0] = KAPPA * (np.eye(4) - orc.gamma(mu))
        w2[2 + 2 * mu, 0, 0] = KAPPA * (np.eye(4) + orc.gamma(mu))
    neumann = W.wl_ptc_create(w1, w2)
    for name, m in (("none", None), ("initial", fresh), ("trained", net), ("neumann", neumann)):
        x = lat.new(W.WL_FULL)
        p = W.wl_pcgnr_params_default()
        p.fallback = 0
        st, info = W.wl_pcgnr_solve(lat.ctx, x, lat.pack(b), KAPPA, m, p)
        xs = lat.unpack(x).reshape(b.shape)
        r = np.linalg.norm(orc.dirac(xs, u, KAPPA, AP) - b) / np.linalg.norm(b)
        assert st == W.WL_OK and r <= 1.05e-10, (name, st, r)
        res[name] = info["iters"]
    print("preconditioned CGNR iterations:", res)
    assert res["trained"] < res["none"] and res["trained"] < res["initial"]
    assert res["neumann"] < res["none"]
    W.wl_ptc_destroy(fresh)
    W.wl_ptc_destroy(neumann)
    lat.close()
