"""Pins of the EigCG oracle (oracle.EigCG): with the search space larger than the
iteration count it is plain CG plus a Rayleigh-Ritz step, so its Ritz values are
the Lanczos ones; over a sequence of right-hand sides the accumulated vectors'
Rayleigh quotients approach the exact lowest eigenvalues of A (dense
eigendecomposition of a tiny lattice's normal operator), and init-CG from them
needs fewer iterations than CG."""

import numpy as np

from oracle import dense
from oracle import oracle as orc
from paper_1405_0700_amd import synth


def setup(dims=(2, 4, 2, 4), kappa=0.124, mu=0.0, seed=850):
    u = synth.su3_links(dims, 0.3, seed)
    ph = (1, 1, 1, -1)
    shape = dims[::-1] + (4, 3)
    m = lambda v: orc.dirac_tm(v.reshape(shape), u, kappa, mu, ph).ravel()
    md = lambda v: orc.dirac_tm(v.reshape(shape), u, kappa, mu, ph, dagger=True).ravel()
    a = lambda v: md(m(v))
    n = 12 * synth.volume(dims)
    D = np.eye(n) - kappa * dense.hopping_matrix(u, ph)
    return a, D.conj().T @ D, n, dims


def test_plain_cg_iterates_and_solution():
    a, A, n, dims = setup()
    b = synth.gaussian_spinor(dims, seed=851).ravel()
    e = orc.EigCG(a, nev=4, m=400, max_vectors=0)
    x, it = e.solve(b, tol=1e-10, collect=False)
    assert np.linalg.norm(A @ x - b) <= 1.01e-10 * np.linalg.norm(b)
    x_cg, info = orc.cg(a, b, tol=1e-10)
    assert abs(info["iters"] - it) <= 0 and np.linalg.norm(x - x_cg) < 1e-12 * np.linalg.norm(x_cg)


def test_ritz_values_approach_the_lowest_eigenvalues():
    a, A, n, dims = setup()
    lam = np.linalg.eigvalsh(A)
    e = orc.EigCG(a, nev=4, m=24, max_vectors=40)
    its = []
    for k in range(8):
        b = synth.gaussian_spinor(dims, seed=860 + k).ravel()
        x, it = e.solve(b, tol=1e-10)
        its.append(it)
        assert np.linalg.norm(A @ x - b) <= 1.01e-10 * np.linalg.norm(b)
    U = np.stack(e.U, axis=1)
    H = U.conj().T @ A @ U
    theta = np.linalg.eigvalsh(H)
    # the lowest Ritz values from the deflation space match the exact lowest eigenvalues
    assert np.all(np.abs(theta[:4] - lam[:4]) <= 1e-6 * lam[:4]), (theta[:4], lam[:4])
    # Rayleigh-Ritz values never go below the true eigenvalues (Cauchy interlacing)
    assert np.all(theta[:8] >= lam[:8] * (1 - 1e-12))
    # deflation pays off: later right-hand sides need fewer iterations than the first
    assert its[-1] < 0.9 * its[0], its


def test_ritz_values_of_the_unrestarted_space_match_a_dense_krylov_projection():
    """Without restarts (m larger than the iteration count) CG's normalised residuals span the
    Krylov space K_k(A, b), so the kept vectors are the lowest Ritz vectors of A on that space:
    their Rayleigh quotients equal the lowest eigenvalues of Q^+ A Q for an orthonormal basis Q
    of K_k(A, b), built here by a dense Lanczos with full reorthogonalisation."""
    a, A, n, dims = setup()
    b = synth.gaussian_spinor(dims, seed=870).ravel()
    e = orc.EigCG(a, nev=3, m=500, max_vectors=3)
    _, k = e.solve(b, tol=1e-6)
    assert len(e.ritz) == 3 and 10 < k < n
    Q = np.zeros((n, k), dtype=np.complex128)
    Q[:, 0] = b / np.linalg.norm(b)
    for j in range(1, k):
        w = A @ Q[:, j - 1]
        for _ in range(2):
            w -= Q[:, :j] @ (Q[:, :j].conj().T @ w)
        Q[:, j] = w / np.linalg.norm(w)
    theta = np.linalg.eigvalsh(Q.conj().T @ A @ Q)
    assert np.allclose(e.ritz, theta[:3], rtol=1e-7), (e.ritz, theta[:3])
    # and they lie above the exact eigenvalues (interlacing)
    lam = np.linalg.eigvalsh(A)
    assert np.all(np.array(e.ritz) >= lam[:3] * (1 - 1e-12))
