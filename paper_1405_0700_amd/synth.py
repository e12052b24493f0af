"""Seeded synthetic inputs for the Wilson hopping operator and its solvers.

This module only *draws* inputs: gauge links, source spinors and random gauge
rotations.  It holds none of the operator's arithmetic (no spin projection, no
hopping sum, no solver step), so that the CPU oracle and the GPU path can both
take their inputs from it without sharing any of the method.

Conventions (identical for every consumer):

* lattice extents ``dims = (Lx, Ly, Lz, Lt)``; a field is stored in canonical
  lexicographic order with ``x`` fastest, i.e. numpy shape ``(Lt, Lz, Ly, Lx,
  ...)``;
* a gauge field has shape ``(Lt, Lz, Ly, Lx, 4, 3, 3)`` complex128, direction
  index ``mu = 0, 1, 2, 3`` for ``x, y, z, t``, then colour row, colour column;
* a spinor field has shape ``(Lt, Lz, Ly, Lx, 4, 3)`` complex128 (spin, colour).

The paper (Sec. 2) takes the links ``U_mu(x)`` as SU(3) matrices and the
spinors as 4-spin x 3-colour fields; it fixes no distribution.  The links here
are ``exp(i * eps * H)`` with ``H = sum_a omega_a lambda_a / 2`` (Gell-Mann
matrices ``lambda_a``, ``omega_a`` iid standard normal), reunitarised to SU(3);
sources are iid complex Gaussians (real and imaginary parts standard normal).
Draw order follows the array order: t, z, y, x (x fastest), then mu, then the
eight omegas; for spinors site, spin, colour, (re, im).
"""

from __future__ import annotations

import numpy as np

__all__ = [
    "gell_mann",
    "su3_links",
    "unit_links",
    "gaussian_spinor",
    "point_source",
    "haar_su3",
    "reunitarise",
    "volume",
    "ptc_weights",
]


def volume(dims) -> int:
    lx, ly, lz, lt = (int(d) for d in dims)
    return lx * ly * lz * lt


def gell_mann() -> np.ndarray:
    """The eight Gell-Mann matrices, shape (8, 3, 3) complex128."""
    lam = np.zeros((8, 3, 3), dtype=np.complex128)
    lam[0][0, 1] = lam[0][1, 0] = 1
    lam[1][0, 1] = -1j
    lam[1][1, 0] = 1j
    lam[2][0, 0] = 1
    lam[2][1, 1] = -1
    lam[3][0, 2] = lam[3][2, 0] = 1
    lam[4][0, 2] = -1j
    lam[4][2, 0] = 1j
    lam[5][1, 2] = lam[5][2, 1] = 1
    lam[6][1, 2] = -1j
    lam[6][2, 1] = 1j
    lam[7][0, 0] = lam[7][1, 1] = 1 / np.sqrt(3)
    lam[7][2, 2] = -2 / np.sqrt(3)
    return lam


def reunitarise(u: np.ndarray) -> np.ndarray:
    """Project (..., 3, 3) near-unitary matrices onto SU(3).

    Row 0 is normalised, row 1 is Gram-Schmidt orthogonalised against it and
    normalised, row 2 is the complex conjugate of the cross product of rows 0
    and 1 (which fixes det = 1).
    """
    u = np.array(u, dtype=np.complex128, copy=True)
    r0 = u[..., 0, :]
    r0 /= np.linalg.norm(r0, axis=-1, keepdims=True)
    r1 = u[..., 1, :]
    proj = np.sum(np.conj(r0) * r1, axis=-1, keepdims=True)
    r1 -= proj * r0
    r1 /= np.linalg.norm(r1, axis=-1, keepdims=True)
    u[..., 0, :] = r0
    u[..., 1, :] = r1
    u[..., 2, :] = np.conj(np.cross(r0, r1))
    return u


def _expi_hermitian(h: np.ndarray, eps: float) -> np.ndarray:
    """exp(i * eps * h) for a batch of Hermitian 3x3 matrices (eigendecomposition)."""
    w, q = np.linalg.eigh(h)
    ph = np.exp(1j * eps * w)
    return np.einsum("...ij,...j,...kj->...ik", q, ph, np.conj(q))


def su3_links(dims, eps: float, seed: int, chunk_sites: int = 1 << 18) -> np.ndarray:
    """Seeded SU(3) gauge field ``U_mu(x) = exp(i eps H_mu(x))``.

    Returns shape ``(Lt, Lz, Ly, Lx, 4, 3, 3)`` complex128.  ``eps = 0`` gives
    the unit gauge field.
    """
    lx, ly, lz, lt = (int(d) for d in dims)
    vol = lx * ly * lz * lt
    rng = np.random.default_rng(seed)
    omega = rng.standard_normal((vol, 4, 8))
    lam_half = gell_mann() / 2.0
    out = np.empty((vol, 4, 3, 3), dtype=np.complex128)
    for s0 in range(0, vol, chunk_sites):
        s1 = min(vol, s0 + chunk_sites)
        h = np.einsum("sma,aij->smij", omega[s0:s1], lam_half)
        out[s0:s1] = reunitarise(_expi_hermitian(h, eps))
    return out.reshape(lt, lz, ly, lx, 4, 3, 3)


def unit_links(dims) -> np.ndarray:
    lx, ly, lz, lt = (int(d) for d in dims)
    u = np.zeros((lt, lz, ly, lx, 4, 3, 3), dtype=np.complex128)
    u[..., 0, 0] = u[..., 1, 1] = u[..., 2, 2] = 1.0
    return u


def gaussian_spinor(dims, seed: int, nsites: int | None = None) -> np.ndarray:
    """Seeded complex Gaussian spinor field, shape (Lt, Lz, Ly, Lx, 4, 3).

    With ``nsites`` given, returns a flat ``(nsites, 4, 3)`` field instead (used
    for one parity of an even/odd ordered lattice).
    """
    rng = np.random.default_rng(seed)
    if nsites is None:
        lx, ly, lz, lt = (int(d) for d in dims)
        shape = (lt, lz, ly, lx, 4, 3)
    else:
        shape = (int(nsites), 4, 3)
    z = rng.standard_normal(shape + (2,))
    return z[..., 0] + 1j * z[..., 1]


def point_source(dims, spin: int, colour: int, site=(0, 0, 0, 0)) -> np.ndarray:
    """Unit point source delta_{x,site} e_spin (x) e_colour; site given as (x, y, z, t)."""
    lx, ly, lz, lt = (int(d) for d in dims)
    f = np.zeros((lt, lz, ly, lx, 4, 3), dtype=np.complex128)
    x, y, z, t = site
    f[t, z, y, x, spin, colour] = 1.0
    return f


def haar_su3(shape, seed: int) -> np.ndarray:
    """Haar-random SU(3) matrices of the given batch shape (QR of a complex Gaussian)."""
    rng = np.random.default_rng(seed)
    z = rng.standard_normal(tuple(shape) + (3, 3, 2))
    z = z[..., 0] + 1j * z[..., 1]
    q, r = np.linalg.qr(z)
    d = np.diagonal(r, axis1=-2, axis2=-1)
    q = q * (d / np.abs(d))[..., None, :]
    det = np.linalg.det(q)
    q = q / (det ** (1.0 / 3.0))[..., None, None]
    return q


def ptc_weights(channels: int, seed: int):
    """Seeded initial weights of the two-layer PTC network (1 -> channels -> 1).

    Shapes (9, channels, 1, 4, 4) and (9, 1, channels, 4, 4) complex128; every
    entry complex Gaussian with standard deviation 0.1 / sqrt(9 C_in), except the
    identity-path matrix of channel 0 in both layers, which is the 4x4 unit
    matrix (so the network starts close to the identity map)."""
    rng = np.random.default_rng(seed)

    def draw(cout, cin):
        sd = 0.1 / np.sqrt(9 * cin)
        z = rng.standard_normal((9, cout, cin, 4, 4, 2)) * sd / np.sqrt(2.0)
        return z[..., 0] + 1j * z[..., 1]

    w1 = draw(channels, 1)
    w2 = draw(1, channels)
    w1[0, 0, 0] = np.eye(4)
    w2[0, 0, 0] = np.eye(4)
    return w1, w2
