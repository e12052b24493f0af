"""Pins of the twisted-mass oracle (oracle.dirac_tm, schur_tm, eo_prepare_tm,
eo_reconstruct_tm) against independent facts: the dense matrix assembled from
Pauli-built gamma matrices plus the diagonal 2 i kappa mu gamma_5 term, the
adjoint identity, gamma_5-hermiticity with mu -> -mu, the free-field closed form
of D_tm^+ D_tm on a plane wave, and the even/odd solve reproducing a dense
solve.  mu = 0 reduces every function to its Wilson counterpart."""

import numpy as np
import pytest

from oracle import dense
from oracle import oracle as orc
from paper_1405_0700_amd import synth


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def random_phases(seed):
    rng = np.random.default_rng(seed)
    return np.exp(1j * rng.uniform(0, 2 * np.pi, 4))


def dense_gamma5():
    gx, gy, gz, gt = dense.chiral_gammas()
    return gt @ gx @ gy @ gz


def dense_dtm(u, kappa, mu, ph, dagger=False):
    vol = synth.volume((u.shape[3], u.shape[2], u.shape[1], u.shape[0]))
    g5 = np.kron(np.eye(vol), np.kron(dense_gamma5(), np.eye(3)))
    nu = (-2.0 if dagger else 2.0) * kappa * mu
    return np.eye(12 * vol) + 1j * nu * g5 - kappa * dense.hopping_matrix(u, ph, dagger)


@pytest.mark.parametrize("dagger", [False, True])
def test_dirac_tm_equals_dense_matrix(dagger):
    dims = (2, 4, 2, 4)
    u = synth.su3_links(dims, 0.6, seed=801)
    ph = random_phases(802)
    phi = synth.gaussian_spinor(dims, seed=803)
    kappa, mu = 0.13, 0.37
    want = (dense_dtm(u, kappa, mu, ph, dagger) @ phi.ravel()).reshape(phi.shape)
    assert rel(orc.dirac_tm(phi, u, kappa, mu, ph, dagger), want) < 1e-14


def test_adjoint_and_gamma5_hermiticity():
    dims = (4, 2, 4, 4)
    u = synth.su3_links(dims, 0.7, seed=804)
    ph = random_phases(805)
    kappa, mu = 0.12, 0.25
    chi = synth.gaussian_spinor(dims, seed=806)
    phi = synth.gaussian_spinor(dims, seed=807)
    lhs = orc.dot(chi, orc.dirac_tm(phi, u, kappa, mu, ph))
    rhs = orc.dot(orc.dirac_tm(chi, u, kappa, mu, ph, dagger=True), phi)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)
    g5 = lambda f: np.einsum("st,...tc->...sc", orc.gamma5(), f)
    # D_tm(mu)^+ = gamma_5 D_tm(-mu) gamma_5
    assert rel(g5(orc.dirac_tm(g5(phi), u, kappa, -mu, ph)), orc.dirac_tm(phi, u, kappa, mu, ph, dagger=True)) < 1e-14


def test_mu_zero_is_wilson():
    dims = (4, 4, 2, 4)
    u = synth.su3_links(dims, 0.5, seed=808)
    ph = random_phases(809)
    phi = synth.gaussian_spinor(dims, seed=810)
    assert np.array_equal(orc.dirac_tm(phi, u, 0.13, 0.0, ph), orc.dirac(phi, u, 0.13, ph))
    pe, po = orc.eo_split(phi, dims)
    assert rel(orc.schur_tm(pe, u, 0.13, 0.0, ph), orc.schur(pe, u, 0.13, ph)) < 1e-15


@pytest.mark.parametrize("n", [(0, 0, 0, 0), (1, 0, 2, 1), (2, 3, 1, 0)])
def test_free_field_normal_operator_on_a_plane_wave(n):
    """Unit links: D_tm^+ D_tm on a plane wave of momentum p is the number
    (1 - 2 kappa sum cos p)^2 + 4 kappa^2 sum sin^2 p + (2 kappa mu)^2 (gamma_5
    anticommutes with every gamma_mu, so the cross terms cancel)."""
    dims = (4, 6, 4, 8)
    theta = np.array([0.0, 0.0, 0.0, np.pi])
    kappa, mu = 0.11, 0.3
    lx, ly, lz, lt = dims
    p = [(2 * np.pi * n[m] + theta[m]) / dims[m] for m in range(4)]
    t, z, y, x = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly), np.arange(lx), indexing="ij")
    rng = np.random.default_rng(811)
    s = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
    b = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))[..., None, None] * s
    u1 = synth.unit_links(dims)
    zph = np.exp(1j * theta)
    got = orc.dirac_tm(orc.dirac_tm(b, u1, kappa, mu, zph), u1, kappa, mu, zph, dagger=True)
    lam = (1 - 2 * kappa * np.sum(np.cos(p))) ** 2 + 4 * kappa ** 2 * np.sum(np.sin(p) ** 2) + (2 * kappa * mu) ** 2
    assert rel(got, lam * b) < 1e-13


def test_even_odd_solve_reproduces_the_dense_solve():
    dims = (2, 2, 4, 4)
    u = synth.su3_links(dims, 0.6, seed=812)
    ph = random_phases(813)
    kappa, mu = 0.12, 0.2
    b = synth.gaussian_spinor(dims, seed=814)
    x = np.linalg.solve(dense_dtm(u, kappa, mu, ph), b.ravel()).reshape(b.shape)
    xe, xo = orc.eo_split(x, dims)
    be, bo = orc.eo_split(b, dims)
    assert rel(orc.schur_tm(xe, u, kappa, mu, ph), orc.eo_prepare_tm(be, bo, u, kappa, mu, ph)) < 1e-12
    assert rel(orc.eo_reconstruct_tm(xe, bo, u, kappa, mu, ph), xo) < 1e-12
