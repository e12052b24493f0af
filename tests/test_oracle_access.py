"""Pins of the link-spinor oracle (oracle.su3_apply), the isolated kernel of the paper's
addressing experiment: psi(x_i) = U(x_i) phi(x_i)."""

import numpy as np

from oracle import oracle as orc
from paper_1405_0700_amd import synth


def _inputs(n, seed):
    rng = np.random.default_rng(seed)
    u = synth.haar_su3((n,), seed)
    phi = rng.standard_normal((n, 4, 3)) + 1j * rng.standard_normal((n, 4, 3))
    psi = rng.standard_normal((n, 4, 3)) + 1j * rng.standard_normal((n, 4, 3))
    return u, phi, psi


def test_identity_links_copy_phi_at_visited_sites_only():
    n = 20
    _, phi, psi = _inputs(n, 1)
    u = np.broadcast_to(np.eye(3, dtype=complex), (n, 3, 3))
    out = orc.su3_apply(u, phi, psi, [3, 7, 7, 11])
    for x in range(n):
        assert np.array_equal(out[x], phi[x] if x in (3, 7, 11) else psi[x])


def test_matches_explicit_sums_on_a_tiny_case():
    u, phi, psi = _inputs(6, 2)
    out = orc.su3_apply(u, phi, psi, [5, 0, 2])
    for x in (5, 0, 2):
        for s in range(4):
            for a in range(3):
                ref = sum(u[x, a, b] * phi[x, s, b] for b in range(3))
                assert abs(out[x, s, a] - ref) <= 1e-15 * (1 + abs(ref))
    # U, not its transpose or adjoint
    x = 5
    assert not np.allclose(out[x, 0], u[x].T @ phi[x, 0])
    assert not np.allclose(out[x, 0], u[x].conj().T @ phi[x, 0])


def test_special_unitary_links_keep_every_colour_vector_norm():
    n = 64
    u, phi, psi = _inputs(n, 3)
    assert np.allclose(np.linalg.det(u), 1.0, atol=1e-12)
    out = orc.su3_apply(u, phi, psi, range(n))
    assert np.allclose(np.linalg.norm(out, axis=-1), np.linalg.norm(phi, axis=-1), rtol=1e-13)
    # and U^+ undoes it
    back = np.einsum("xba,xsb->xsa", u.conj(), out)
    assert np.allclose(back, phi, atol=1e-13)


def test_visit_order_does_not_matter_for_a_permutation():
    n = 50
    u, phi, psi = _inputs(n, 4)
    perm = np.random.default_rng(5).permutation(n)
    assert np.array_equal(orc.su3_apply(u, phi, psi, perm), orc.su3_apply(u, phi, psi, range(n)))
