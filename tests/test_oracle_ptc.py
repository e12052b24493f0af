"""Pins of the PTC-network oracle (oracle/ptc.py) against independent facts:
the Wilson hopping term (the C oracle of Eq. (1)) as a special case, the
identity, transport inverses, gauge equivariance, the adjoint identity,
central finite differences of the loss, and the first Adam step."""

import numpy as np
import pytest

from oracle import oracle as orc
from oracle import dense, ptc
from paper_1405_0700_amd import synth

AP = (1, 1, 1, -1)


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel())


def random_phases(seed):
    rng = np.random.default_rng(seed)
    return np.exp(1j * rng.uniform(0, 2 * np.pi, 4))


def random_weights(cout, cin, seed):
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((ptc.NPATH, cout, cin, 4, 4, 2))
    return z[..., 0] + 1j * z[..., 1]


def test_special_weights_reproduce_the_hopping_term():
    dims = (4, 2, 4, 6)
    u = synth.su3_links(dims, 0.7, seed=1)
    ph = random_phases(2)
    phi = synth.gaussian_spinor(dims, seed=3)
    w = np.zeros((ptc.NPATH, 1, 1, 4, 4), dtype=np.complex128)
    for mu in range(4):
        g = orc.gamma(mu)
        w[1 + 2 * mu, 0, 0] = np.eye(4) - g
        w[2 + 2 * mu, 0, 0] = np.eye(4) + g
    out = ptc.layer([phi], w, u, ph)[0]
    assert rel(out, orc.hop(phi, u, ph)) < 1e-14


def test_identity_weights():
    dims = (2, 4, 2, 4)
    u = synth.su3_links(dims, 0.7, seed=4)
    phi = synth.gaussian_spinor(dims, seed=5)
    w = np.zeros((ptc.NPATH, 1, 1, 4, 4), dtype=np.complex128)
    w[0, 0, 0] = np.eye(4)
    assert np.array_equal(ptc.layer([phi], w, u, AP)[0], phi)
    w1, w2 = synth.ptc_weights(8, seed=6)
    w1[:, 1:] = 0
    w1[1:, 0] = 0
    w2[:, :, 1:] = 0
    w2[1:] = 0
    out, _ = ptc.net_apply(phi, w1, w2, u, AP)
    assert np.array_equal(out, phi)


@pytest.mark.parametrize("mu", range(4))
def test_forward_and_backward_transports_are_inverse(mu):
    dims = (4, 4, 2, 4)
    u = synth.su3_links(dims, 0.9, seed=7)
    ph = random_phases(8)
    phi = synth.gaussian_spinor(dims, seed=9)
    fwd, bwd = 1 + 2 * mu, 2 + 2 * mu
    back = ptc.transport(ptc.transport(phi, u, ph, bwd), u, ph, fwd)
    assert rel(back, phi) < 1e-14
    assert ptc.reverse_path(fwd) == bwd and ptc.reverse_path(bwd) == fwd


def gauge_transform(u, omega):
    out = np.empty_like(u)
    for mu in range(4):
        om_fwd = np.roll(omega, -1, axis=ptc._AXIS[mu])
        out[..., mu, :, :] = omega @ u[..., mu, :, :] @ np.conj(np.swapaxes(om_fwd, -1, -2))
    return out


def test_network_is_gauge_equivariant():
    dims = (4, 2, 2, 4)
    u = synth.su3_links(dims, 0.8, seed=10)
    ph = random_phases(11)
    w1, w2 = random_weights(3, 1, 12), random_weights(1, 3, 13)
    r = synth.gaussian_spinor(dims, seed=14)
    omega = synth.haar_su3((dims[3], dims[2], dims[1], dims[0]), seed=15)
    rot = lambda f: np.einsum("...ij,...sj->...si", omega, f)
    lhs, _ = ptc.net_apply(rot(r), w1, w2, gauge_transform(u, omega), ph)
    rhs, _ = ptc.net_apply(r, w1, w2, u, ph)
    assert rel(lhs, rot(rhs)) < 1e-13


def test_layer_adjoint_identity():
    dims = (2, 4, 2, 4)
    u = synth.su3_links(dims, 0.8, seed=16)
    ph = random_phases(17)
    w = random_weights(3, 2, 18)
    ins = [synth.gaussian_spinor(dims, seed=20 + b) for b in range(2)]
    chis = [synth.gaussian_spinor(dims, seed=30 + a) for a in range(3)]
    lhs = sum(np.vdot(c, o) for c, o in zip(chis, ptc.layer(ins, w, u, ph)))
    rhs = sum(np.vdot(g, i) for g, i in zip(ptc.layer_adjoint(chis, w, u, ph), ins))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_gradients_match_central_finite_differences():
    dims = (2, 2, 2, 4)
    u = synth.su3_links(dims, 0.6, seed=40)
    ph = random_phases(41)
    w1, w2 = random_weights(2, 1, 42) * 0.3, random_weights(1, 2, 43) * 0.3
    pairs = [(synth.gaussian_spinor(dims, seed=50 + i), synth.gaussian_spinor(dims, seed=60 + i)) for i in range(2)]
    loss, g1, g2 = ptc.loss_and_grads(pairs, w1, w2, u, ph)
    assert loss > 0
    rng = np.random.default_rng(7)
    eps = 1e-6
    for which, w, g in (("w1", w1, g1), ("w2", w2, g2)):
        for _ in range(6):
            k = tuple(rng.integers(0, n) for n in w.shape)
            for unit, part in ((1.0, "re"), (1j, "im")):
                wp, wm = w.copy(), w.copy()
                wp[k] += unit * eps
                wm[k] -= unit * eps
                args_p = (wp, w2) if which == "w1" else (w1, wp)
                args_m = (wm, w2) if which == "w1" else (w1, wm)
                fd = (ptc.loss_and_grads(pairs, *args_p, u, ph)[0] - ptc.loss_and_grads(pairs, *args_m, u, ph)[0]) / (2 * eps)
                want = 2 * (g[k].real if part == "re" else g[k].imag)
                assert abs(fd - want) <= 1e-7 * max(1.0, abs(want)), (which, k, part, fd, want)


def test_residual_loss_gradients_match_central_finite_differences():
    dims = (2, 2, 4, 2)
    u = synth.su3_links(dims, 0.6, seed=44)
    ph = random_phases(45)
    w1, w2 = random_weights(2, 1, 46) * 0.3, random_weights(1, 2, 47) * 0.3
    rs = [synth.gaussian_spinor(dims, seed=70 + i) for i in range(2)]
    kappa = 0.11
    loss, g1, g2 = ptc.loss_and_grads_residual(rs, w1, w2, u, ph, kappa)
    # the loss is the definition written out with the dense matrix of D
    dm = np.eye(12 * synth.volume(dims)) - kappa * dense.hopping_matrix(u, ph)
    want = np.mean([np.linalg.norm(dm @ ptc.net_apply(r, w1, w2, u, ph)[0].ravel() - r.ravel()) ** 2
                    / np.linalg.norm(r) ** 2 for r in rs])
    assert abs(loss - want) < 1e-12 * want
    rng = np.random.default_rng(8)
    eps = 1e-6
    for which, w, g in (("w1", w1, g1), ("w2", w2, g2)):
        for _ in range(5):
            k = tuple(rng.integers(0, n) for n in w.shape)
            for unit, part in ((1.0, "re"), (1j, "im")):
                wp, wm = w.copy(), w.copy()
                wp[k] += unit * eps
                wm[k] -= unit * eps
                args_p = (wp, w2) if which == "w1" else (w1, wp)
                args_m = (wm, w2) if which == "w1" else (w1, wm)
                fd = (ptc.loss_and_grads_residual(rs, *args_p, u, ph, kappa)[0]
                      - ptc.loss_and_grads_residual(rs, *args_m, u, ph, kappa)[0]) / (2 * eps)
                want = 2 * (g[k].real if part == "re" else g[k].imag)
                assert abs(fd - want) <= 1e-7 * max(1.0, abs(want)), (which, k, part, fd, want)


def test_first_adam_step_moves_each_parameter_by_lr():
    rng = np.random.default_rng(3)
    w = rng.standard_normal((5, 4)) + 1j * rng.standard_normal((5, 4))
    g = rng.standard_normal((5, 4)) + 1j * rng.standard_normal((5, 4))
    m = np.zeros(w.shape + (2,))
    v = np.zeros(w.shape + (2,))
    w2, m, v = ptc.adam_step(w, g, m, v, t=1, lr=1e-3, eps=0.0)
    d = w2 - w
    # bias-corrected first step: -lr * sign of the real-parameter gradient (2 Re G, 2 Im G)
    assert np.allclose(d.real, -1e-3 * np.sign(g.real), atol=1e-15)
    assert np.allclose(d.imag, -1e-3 * np.sign(g.imag), atol=1e-15)


def test_init_weights_shapes_and_pass_through():
    w1, w2 = synth.ptc_weights(8, seed=530)
    assert w1.shape == (9, 8, 1, 4, 4) and w2.shape == (9, 1, 8, 4, 4)
    assert np.array_equal(w1[0, 0, 0], np.eye(4)) and np.array_equal(w2[0, 0, 0], np.eye(4))
    sd = np.std(np.concatenate([w1[1:].ravel(), w1[0, 1:].ravel()]))
    assert abs(sd - 0.1 / 3.0) < 0.01


def test_adam_with_a_constant_gradient_steps_lr_against_its_sign_every_step():
    """Adam's bias corrections make the moments of a constant gradient exact at every step t:
    m_t / (1 - b1^t) = g and v_t / (1 - b2^t) = g^2, so (eps = 0) every step moves each real parameter by
    exactly lr against the sign of its gradient, and after T steps w_T = w_0 - T lr sign(g).  A dropped or
    wrong bias correction, or moments that restart every step, breaks this after the first step."""
    rng = np.random.default_rng(5)
    w0 = rng.standard_normal((3, 4)) + 1j * rng.standard_normal((3, 4))
    g = rng.standard_normal((3, 4)) + 1j * rng.standard_normal((3, 4))  # dL/dW*: real gradient (2 Re, 2 Im)
    w, m, v = w0.copy(), np.zeros((3, 4, 2)), np.zeros((3, 4, 2))
    lr, T = 1e-2, 7
    for t in range(1, T + 1):
        w, m, v = ptc.adam_step(w, g, m, v, t, lr=lr, eps=0.0)
        want = w0 - t * lr * (np.sign(g.real) + 1j * np.sign(g.imag))
        assert np.allclose(w, want, rtol=0, atol=1e-13), t
        # the raw moments carry over: m_t = (1 - b1^t) 2 Re/Im g, v_t = (1 - b2^t) (2 Re/Im g)^2
        gr = np.stack([2 * g.real, 2 * g.imag], axis=-1)
        assert np.allclose(m, (1 - 0.9 ** t) * gr, rtol=1e-13, atol=0)
        assert np.allclose(v, (1 - 0.999 ** t) * gr * gr, rtol=1e-12, atol=0)
