"""Dense-matrix assembler of the hopping term -- TEST INFRASTRUCTURE ONLY.

A second, independent CPU oracle for tiny lattices: it builds the
12V x 12V complex matrix of H (paper Sec. 2, Eq. (1)) block by block from
Kronecker products (spin matrix) x (colour matrix), with the gamma matrices
*constructed* from the Pauli matrices rather than typed in:

    gamma_mu = [[0, A_mu], [A_mu^+, 0]],   A = (-i s1, -i s2, -i s3, -1)

(chiral basis, mu = x, y, z, t).  It shares no code with ``wilson_oracle.c``;
agreement between the two pins the typed-in gamma table, the neighbour
indexing, the boundary phases and the projector signs of both.

Row/column index of a field component: (lex * 4 + spin) * 3 + colour, with
lex = x + Lx (y + Ly (z + Lz t)).
"""

from __future__ import annotations

import numpy as np

SIGMA = [
    np.array([[0, 1], [1, 0]], dtype=np.complex128),
    np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
    np.array([[1, 0], [0, -1]], dtype=np.complex128),
]


def chiral_gammas():
    """gamma_x, gamma_y, gamma_z, gamma_t built from Pauli blocks."""
    blocks = [-1j * SIGMA[0], -1j * SIGMA[1], -1j * SIGMA[2], -np.eye(2, dtype=np.complex128)]
    out = []
    for a in blocks:
        g = np.zeros((4, 4), dtype=np.complex128)
        g[0:2, 2:4] = a
        g[2:4, 0:2] = a.conj().T
        out.append(g)
    return out


def hopping_matrix(gauge: np.ndarray, phases, dagger: bool = False) -> np.ndarray:
    """Dense H (or H^+ if dagger) for a canonical gauge field (tiny lattices only)."""
    lt, lz, ly, lx = gauge.shape[:4]
    L = (lx, ly, lz, lt)
    vol = lx * ly * lz * lt
    g = gauge.reshape(vol, 4, 3, 3)
    z = np.asarray(phases, dtype=np.complex128).reshape(4)
    gam = chiral_gammas()
    one = np.eye(4, dtype=np.complex128)
    s = -1.0 if dagger else 1.0
    h = np.zeros((12 * vol, 12 * vol), dtype=np.complex128)

    def lex(c):
        return c[0] + L[0] * (c[1] + L[1] * (c[2] + L[2] * c[3]))

    for site in range(vol):
        c = [site % L[0], (site // L[0]) % L[1], (site // (L[0] * L[1])) % L[2],
             site // (L[0] * L[1] * L[2])]
        rows = slice(12 * site, 12 * site + 12)
        for mu in range(4):
            # forward hop: (1 - s gamma_mu) (x) U_mu(x), times z_mu if it wraps
            cf = list(c)
            cf[mu] += 1
            ph = 1.0
            if cf[mu] == L[mu]:
                cf[mu] = 0
                ph = z[mu]
            nf = lex(cf)
            h[rows, 12 * nf:12 * nf + 12] += ph * np.kron(one - s * gam[mu], g[site, mu])
            # backward hop: (1 + s gamma_mu) (x) U_mu(x - mu)^+, times conj(z_mu) if it wraps
            cb = list(c)
            cb[mu] -= 1
            ph = 1.0
            if cb[mu] < 0:
                cb[mu] = L[mu] - 1
                ph = np.conj(z[mu])
            nb = lex(cb)
            h[rows, 12 * nb:12 * nb + 12] += ph * np.kron(one + s * gam[mu], g[nb, mu].conj().T)
    return h


def as_vector(field: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(field).reshape(-1)
