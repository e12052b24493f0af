"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

None of these tests retypes the oracle's formula: each checks it against an
independent construction (the dense assembler, a hand-worked example, a closed
form, an identity or an invariant), chosen so that a dropped term, a wrong
sign or index, or a transposed operand fails at least one of them.
"""

import os

import numpy as np
import pytest

from oracle import dense
from oracle import oracle as orc
from paper_1405_0700_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
AP = (1, 1, 1, -1)  # periodic in space, antiperiodic in time


def rel(a, b):
    return np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300)


def random_phases(seed):
    rng = np.random.default_rng(seed)
    return np.exp(1j * rng.uniform(0, 2 * np.pi, 4))


# ---------------------------------------------------------------- gammas
def test_gamma_clifford_and_hermitian():
    g = [orc.gamma(mu) for mu in range(4)]
    for mu in range(4):
        assert np.allclose(g[mu], g[mu].conj().T, atol=0)
        for nu in range(4):
            anti = g[mu] @ g[nu] + g[nu] @ g[mu]
            assert np.allclose(anti, 2 * np.eye(4) * (mu == nu), atol=0)
    assert np.allclose(orc.gamma5(), np.diag([1, 1, -1, -1]), atol=0)


def test_gamma_table_equals_pauli_construction():
    built = dense.chiral_gammas()
    for mu in range(4):
        assert np.array_equal(orc.gamma(mu), built[mu])


@pytest.mark.parametrize("mu", range(4))
@pytest.mark.parametrize("sign", [+1, -1])
def test_half_spinor_structure(mu, sign):
    """After Eq. (2): the lower two spin components of (1 -/+ gamma_mu) phi
    follow from the upper two.  In the chiral basis the lower rows equal
    -/+ A_mu^+ times the upper rows, checked on all 4 spin basis vectors."""
    p = np.eye(4) - sign * orc.gamma(mu)
    a = orc.gamma(mu)[0:2, 2:4]  # A_mu
    for col in range(4):
        e = np.zeros(4, complex)
        e[col] = 1
        v = p @ e
        assert np.allclose(v[2:4], -sign * a.conj().T @ v[0:2], atol=1e-15)
    assert np.linalg.matrix_rank(p) == 2


# ---------------------------------------------------------------- H vs dense
@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (2, 4, 2, 6)])
@pytest.mark.parametrize("dagger", [False, True])
def test_hop_equals_dense_matrix(dims, dagger):
    u = synth.su3_links(dims, 0.7, seed=11)
    ph = random_phases(3)
    phi = synth.gaussian_spinor(dims, seed=12)
    h = dense.hopping_matrix(u, ph, dagger=dagger)
    want = (h @ dense.as_vector(phi)).reshape(phi.shape)
    got = orc.hop(phi, u, ph, dagger=dagger)
    assert rel(got, want) < 1e-14


def test_dense_dagger_is_conjugate_transpose():
    dims = (2, 2, 2, 4)
    u = synth.su3_links(dims, 0.9, seed=5)
    ph = random_phases(9)
    h = dense.hopping_matrix(u, ph)
    hd = dense.hopping_matrix(u, ph, dagger=True)
    assert np.allclose(hd, h.conj().T, atol=1e-14)


def test_golden_point_source():
    dims = (4, 4, 4, 4)
    u = synth.unit_links(dims)
    phi = synth.point_source(dims, 0, 0)
    psi = orc.hop(phi, u, AP)
    want = np.zeros_like(psi)
    rows = np.loadtxt(os.path.join(GOLDEN, "free_point_source_4444.txt"))
    for x, y, z, t, s, re, im in rows:
        want[int(t), int(z), int(y), int(x), int(s), 0] = re + 1j * im
    assert np.array_equal(psi, want)


# ---------------------------------------------------------------- closed forms
def plane_wave(dims, n, theta, u):
    lx, ly, lz, lt = dims
    p = [(2 * np.pi * n[m] + theta[m]) / dims[m] for m in range(4)]
    t, z, y, x = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly), np.arange(lx), indexing="ij")
    ph = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))
    return ph[..., None, None] * u[None, None, None, None], np.array(p)


@pytest.mark.parametrize("n", [(0, 0, 0, 0), (1, 2, 0, 3), (3, 1, 2, 5)])
def test_free_field_plane_wave(n):
    dims = (4, 6, 4, 8)
    theta = np.array([0.3, 0.0, -1.1, np.pi])
    rng = np.random.default_rng(1)
    u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
    phi, p = plane_wave(dims, n, theta, u)
    psi = orc.hop(phi, synth.unit_links(dims), np.exp(1j * theta))
    spin = 2 * np.sum(np.cos(p)) * np.eye(4) - 2j * sum(dense.chiral_gammas()[m] * np.sin(p[m]) for m in range(4))
    want = np.einsum("ab,...bc->...ac", spin, phi)
    assert rel(psi, want) < 1e-14


# ---------------------------------------------------------------- identities
@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (2, 2, 4, 2)])
def test_adjoint_identity(dims):
    u = synth.su3_links(dims, 0.5, seed=21)
    ph = random_phases(22)
    chi = synth.gaussian_spinor(dims, seed=23)
    phi = synth.gaussian_spinor(dims, seed=24)
    lhs = orc.dot(chi, orc.hop(phi, u, ph))
    rhs = orc.dot(orc.hop(chi, u, ph, dagger=True), phi)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def test_gamma5_hermiticity():
    dims = (4, 4, 2, 6)
    u = synth.su3_links(dims, 0.5, seed=31)
    ph = random_phases(32)
    phi = synth.gaussian_spinor(dims, seed=33)
    g5 = np.diag([1.0, 1.0, -1.0, -1.0])
    lhs = orc.hop(phi, u, ph, dagger=True)
    rhs = np.einsum("ab,...bc->...ac", g5, orc.hop(np.einsum("ab,...bc->...ac", g5, phi), u, ph))
    assert rel(lhs, rhs) < 1e-15


def test_linearity():
    dims = (4, 2, 2, 4)
    u = synth.su3_links(dims, 0.5, seed=41)
    a = synth.gaussian_spinor(dims, seed=42)
    b = synth.gaussian_spinor(dims, seed=43)
    c = 0.3 - 1.7j
    lhs = orc.hop(a + c * b, u, AP)
    rhs = orc.hop(a, u, AP) + c * orc.hop(b, u, AP)
    assert rel(lhs, rhs) < 1e-14


def gauge_transform(u, omega):
    """U_mu(x) -> Omega(x) U_mu(x) Omega(x + mu)^+ (periodic shift)."""
    out = np.empty_like(u)
    axes = {0: 3, 1: 2, 2: 1, 3: 0}  # mu -> array axis of (t, z, y, x)
    for mu in range(4):
        om_fwd = np.roll(omega, -1, axis=axes[mu])
        out[..., mu, :, :] = omega @ u[..., mu, :, :] @ np.conj(np.swapaxes(om_fwd, -1, -2))
    return out


@pytest.mark.parametrize("dagger", [False, True])
def test_gauge_covariance(dagger):
    dims = (4, 4, 2, 4)
    u = synth.su3_links(dims, 0.8, seed=51)
    ph = random_phases(52)
    omega = synth.haar_su3((dims[3], dims[2], dims[1], dims[0]), seed=53)
    phi = synth.gaussian_spinor(dims, seed=54)
    ug = gauge_transform(u, omega)
    phig = np.einsum("...ij,...sj->...si", omega, phi)
    lhs = orc.hop(phig, ug, ph, dagger=dagger)
    rhs = np.einsum("...ij,...sj->...si", omega, orc.hop(phi, u, ph, dagger=dagger))
    assert rel(lhs, rhs) < 1e-14


def test_even_odd_structure_and_spectrum():
    dims = (2, 2, 2, 4)
    u = synth.su3_links(dims, 0.6, seed=61)
    ph = random_phases(62)
    e = synth.gaussian_spinor(dims, seed=63)
    par = orc.parity_mask(dims)
    e[par == 1] = 0
    out = orc.hop(e, u, ph)
    assert np.all(out[par == 0] == 0)  # H_ee = 0
    h = dense.hopping_matrix(u, ph)
    ev = np.linalg.eigvals(h)
    # H anticommutes with the parity sign -> spectrum symmetric under lambda -> -lambda
    def set_distance(a, b):
        return np.abs(a[:, None] - b[None, :]).min(axis=1).max()

    assert set_distance(ev, -ev) < 1e-10
    # gamma5-hermiticity -> eigenvalues come in complex-conjugate pairs
    assert set_distance(ev, np.conj(ev)) < 1e-10


def test_eo_split_matches_lex_ranking():
    dims = (4, 2, 2, 2)
    f = synth.gaussian_spinor(dims, seed=71)
    e, o = orc.eo_split(f, dims)
    assert e.shape == (16, 4, 3) and o.shape == (16, 4, 3)
    flat = f.reshape(-1, 4, 3)
    lx, ly, lz, lt = dims
    ie = io = 0
    for lex in range(flat.shape[0]):
        x = lex % lx; y = (lex // lx) % ly; z = (lex // (lx * ly)) % lz; t = lex // (lx * ly * lz)
        if (x + y + z + t) % 2 == 0:
            assert np.array_equal(e[ie], flat[lex]); ie += 1
        else:
            assert np.array_equal(o[io], flat[lex]); io += 1
    assert np.array_equal(orc.eo_join(e, o, dims), f)


# ---------------------------------------------------------------- D, D_hat
def test_schur_solution_solves_full_system():
    dims = (2, 2, 2, 4)
    kappa = 0.13
    u = synth.su3_links(dims, 0.5, seed=81)
    b = synth.gaussian_spinor(dims, seed=82)
    b_e, b_o = orc.eo_split(b, dims)
    bh = orc.eo_prepare(b_e, b_o, u, kappa, AP)
    # D_hat as a dense matrix on the even sites, from the oracle's own action
    n = b_e.size
    cols = []
    for k in range(n):
        v = np.zeros(n, complex); v[k] = 1
        cols.append(orc.schur(v.reshape(b_e.shape), u, kappa, AP).ravel())
    mhat = np.stack(cols, axis=1)
    x_e = np.linalg.solve(mhat, bh.ravel()).reshape(b_e.shape)
    x_o = orc.eo_reconstruct(x_e, b_o, u, kappa, AP)
    x = orc.eo_join(x_e, x_o, dims)
    assert rel(orc.dirac(x, u, kappa, AP), b) < 1e-13
    # and D via the dense assembler agrees with the oracle's D
    h = dense.hopping_matrix(u, AP)
    dm = np.eye(h.shape[0]) - kappa * h
    assert rel(dm @ x.ravel(), b.ravel()) < 1e-13


def test_schur_dagger_is_gamma5_conjugate():
    dims = (4, 2, 2, 2)
    u = synth.su3_links(dims, 0.5, seed=91)
    v = synth.gaussian_spinor(dims, seed=92, nsites=16)
    g5 = np.diag([1.0, 1.0, -1.0, -1.0])
    lhs = orc.schur(v, u, 0.12, AP, dagger=True)
    rhs = np.einsum("ab,sbc->sac", g5, orc.schur(np.einsum("ab,sbc->sac", g5, v), u, 0.12, AP))
    assert rel(lhs, rhs) < 1e-15


# ---------------------------------------------------------------- CG
@pytest.mark.parametrize("n", [(0, 0, 0, 0), (1, 0, 2, 3)])
def test_cg_free_plane_wave_converges_in_one_iteration(n):
    dims = (4, 4, 4, 8)
    kappa = 0.12
    theta = np.array([0.0, 0.0, 0.0, np.pi])
    u1 = synth.unit_links(dims)
    rng = np.random.default_rng(7)
    spin = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
    b, p = plane_wave(dims, n, theta, spin)
    z = np.exp(1j * theta)
    m = lambda v: orc.dirac(v, u1, kappa, z)
    md = lambda v: orc.dirac(v, u1, kappa, z, dagger=True)
    x, info = orc.cg_normal(m, md, b, tol=1e-12)
    lam = (1 - 2 * kappa * np.sum(np.cos(p))) ** 2 + 4 * kappa ** 2 * np.sum(np.sin(p) ** 2)
    assert info["iters"] == 1
    assert rel(x, b / lam) < 1e-13


def test_cg_converges_within_number_of_distinct_eigenvalues():
    dims = (4, 4, 4, 4)
    kappa = 0.1
    theta = np.zeros(4)
    u1 = synth.unit_links(dims)
    rng = np.random.default_rng(8)
    modes = [(0, 0, 0, 0), (1, 0, 0, 0), (1, 1, 0, 0), (2, 1, 1, 0)]  # distinct sum cos p
    b = 0
    for n in modes:
        s = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
        b = b + plane_wave(dims, n, theta, s)[0]
    m = lambda v: orc.dirac(v, u1, kappa, np.ones(4))
    md = lambda v: orc.dirac(v, u1, kappa, np.ones(4), dagger=True)
    x, info = orc.cg_normal(m, md, b, tol=1e-12)
    assert info["iters"] <= len(modes)
    assert info["true_rel_resid"] < 1e-12


def test_cg_matches_dense_solve():
    dims = (2, 2, 2, 4)
    kappa = 0.12
    u = synth.su3_links(dims, 0.5, seed=101)
    b = synth.gaussian_spinor(dims, seed=102)
    m = lambda v: orc.dirac(v, u, kappa, AP)
    md = lambda v: orc.dirac(v, u, kappa, AP, dagger=True)
    x, info = orc.cg_normal(m, md, b, tol=1e-12)
    h = dense.hopping_matrix(u, AP)
    dm = np.eye(h.shape[0]) - kappa * h
    want = np.linalg.solve(dm.conj().T @ dm, b.ravel())
    cond = np.linalg.cond(dm.conj().T @ dm)
    assert rel(x.ravel(), want) < 10 * cond * 1e-12
    assert info["true_rel_resid"] <= 1e-12


def test_cg_fixed_iterations_and_zero_rhs():
    dims = (2, 2, 2, 2)
    u = synth.su3_links(dims, 0.5, seed=111)
    m = lambda v: orc.dirac(v, u, 0.1, AP)
    md = lambda v: orc.dirac(v, u, 0.1, AP, dagger=True)
    b = synth.gaussian_spinor(dims, seed=112)
    _, info = orc.cg_normal(m, md, b, fixed_iters=3)
    assert info["iters"] == 3 and len(info["resid_history"]) == 4
    x, info = orc.cg_normal(m, md, np.zeros_like(b))
    assert info["iters"] == 0 and not np.any(x)


# ---------------------------------------------------------------- generator
def test_generator_links_are_su3():
    u = synth.su3_links((4, 4, 2, 2), 0.5, seed=1).reshape(-1, 3, 3)
    eye = np.eye(3)
    uu = np.einsum("sji,sjk->sik", np.conj(u), u)
    assert np.abs(uu - eye).max() < 1e-14
    assert np.abs(np.linalg.det(u) - 1).max() < 1e-14
    u0 = synth.su3_links((2, 2, 2, 2), 0.0, seed=1)
    assert np.abs(u0 - synth.unit_links((2, 2, 2, 2))).max() < 1e-15


def test_generator_is_seeded():
    a = synth.su3_links((2, 2, 2, 2), 0.2, seed=5)
    b = synth.su3_links((2, 2, 2, 2), 0.2, seed=5)
    c = synth.su3_links((2, 2, 2, 2), 0.2, seed=6)
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    # small eps: 1 - Re tr U / 3 ~ eps^2 <tr H^2> / 6 with <tr H^2> = 4 (8 omegas / 2)
    u = synth.su3_links((8, 8, 8, 8), 0.2, seed=7).reshape(-1, 3, 3)
    plaq = np.mean(np.trace(u, axis1=1, axis2=2).real) / 3
    assert abs((1 - plaq) - 0.04 * 4 / 6) < 2e-3
