"""FP64 CPU oracle of the Wilson operator and its CG solver -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this module.  The product path (the HIP library and
its Python binding) never imports, links or calls it, and the two share no
code: this module builds on ``wilson_oracle.c`` (a literal transcription of
Eq. (1) with full 4x4 spin matrices) and on plain numpy.

Everything here works on canonical fields:
  gauge  : (Lt, Lz, Ly, Lx, 4, 3, 3) complex128
  spinor : (Lt, Lz, Ly, Lx, 4, 3) complex128 (full lattice), or
           (V/2, 4, 3) complex128 for one parity of the even/odd ordered
           lattice, its sites in increasing lexicographic order.

Operators (paper Sec. 2 defines only the hopping term H of Eq. (1); the rest
are the readings listed in the design notes):
  H        hopping term, Eq. (1)                         -> hop()
  H^+      its adjoint (projectors 1 -/+ gamma swapped)  -> hop(dagger=True)
  D        1 - kappa H                                   -> dirac()
  D_hat    1 - kappa^2 H_eo H_oe on even sites           -> schur()
  CG       conjugate gradient on A = M^+ M               -> cg(), cg_normal()

Dot products are plain numpy pairwise sums in FP64.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
import sys
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "wilson_oracle.c")
_LIB = os.path.join(_HERE, "_wilson_oracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile wilson_oracle.c with gcc (OpenMP) into oracle/_wilson_oracle.so."""
    if (not force and os.path.exists(_LIB)
            and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC)):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
           "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    with _lock:
        if _lib is None:
            path = build()
            l = ctypes.CDLL(path)
            dp = ctypes.POINTER(ctypes.c_double)
            ip = ctypes.POINTER(ctypes.c_int)
            l.orc_hopping.argtypes = [dp, dp, dp, ip, dp, ctypes.c_int]
            l.orc_hopping.restype = None
            l.orc_gamma.argtypes = [ctypes.c_int, dp]
            l.orc_gamma.restype = None
            l.orc_max_threads.restype = ctypes.c_int
            l.orc_set_threads.argtypes = [ctypes.c_int]
            _lib = l
    return _lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def max_threads() -> int:
    return int(lib().orc_max_threads())


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


def gamma(mu: int) -> np.ndarray:
    """gamma_mu as used by the oracle (4x4 complex128)."""
    buf = np.zeros(32, dtype=np.float64)
    lib().orc_gamma(int(mu), _dptr(buf))
    return (buf[0::2] + 1j * buf[1::2]).reshape(4, 4)


def gamma5() -> np.ndarray:
    """gamma_5 = gamma_t gamma_x gamma_y gamma_z."""
    return gamma(3) @ gamma(0) @ gamma(1) @ gamma(2)


def phases_array(phases) -> np.ndarray:
    """Boundary phases as 4 complex numbers z_mu (x, y, z, t)."""
    z = np.asarray(phases, dtype=np.complex128).reshape(4)
    return np.ascontiguousarray(np.stack([z.real, z.imag], axis=-1).reshape(8))


def dims_of(gauge: np.ndarray):
    lt, lz, ly, lx = gauge.shape[:4]
    return (lx, ly, lz, lt)


# --------------------------------------------------------------------------
# Hopping term, Eq. (1), full lattice
# --------------------------------------------------------------------------
def hop(phi: np.ndarray, gauge: np.ndarray, phases, dagger: bool = False) -> np.ndarray:
    """H phi (or H^+ phi) on the full lattice, Eq. (1)."""
    dims = dims_of(gauge)
    phi = np.ascontiguousarray(phi, dtype=np.complex128)
    assert phi.shape == gauge.shape[:4] + (4, 3), phi.shape
    g = np.ascontiguousarray(gauge, dtype=np.complex128)
    out = np.empty_like(phi)
    d = (ctypes.c_int * 4)(*dims)
    lib().orc_hopping(_dptr(out.view(np.float64)), _dptr(phi.view(np.float64)),
                      _dptr(g.view(np.float64)), d, _dptr(phases_array(phases)),
                      1 if dagger else 0)
    return out


# --------------------------------------------------------------------------
# Even/odd ordering
# --------------------------------------------------------------------------
def parity_mask(dims) -> np.ndarray:
    """Parity (x+y+z+t) mod 2 of every site, shape (Lt, Lz, Ly, Lx)."""
    lx, ly, lz, lt = dims
    t, z, y, x = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly),
                             np.arange(lx), indexing="ij")
    return (x + y + z + t) % 2


def eo_split(full: np.ndarray, dims):
    """Full canonical spinor -> (even half, odd half), each (V/2, 4, 3)."""
    par = parity_mask(dims)
    return full[par == 0].copy(), full[par == 1].copy()


def eo_join(even: np.ndarray, odd: np.ndarray, dims) -> np.ndarray:
    lx, ly, lz, lt = dims
    par = parity_mask(dims)
    full = np.zeros((lt, lz, ly, lx, 4, 3), dtype=np.complex128)
    full[par == 0] = even
    full[par == 1] = odd
    return full


def hop_eo(phi_half: np.ndarray, in_parity: int, gauge, phases, dagger=False) -> np.ndarray:
    """H_{1-p, p} phi_p: hopping term from parity ``in_parity`` to the other one.

    Computed by embedding the half field into an otherwise zero full field,
    applying the full-lattice H and keeping the other parity.
    """
    dims = dims_of(gauge)
    zero = np.zeros_like(phi_half)
    full = eo_join(phi_half, zero, dims) if in_parity == 0 else eo_join(zero, phi_half, dims)
    out = hop(full, gauge, phases, dagger)
    e, o = eo_split(out, dims)
    return o if in_parity == 0 else e


# --------------------------------------------------------------------------
# Dirac operators built on H
# --------------------------------------------------------------------------
def dirac(phi, gauge, kappa, phases, dagger=False):
    """D phi = phi - kappa H phi (D^+ with H^+), full lattice."""
    return phi - kappa * hop(phi, gauge, phases, dagger)


def twist(phi, nu):
    """(1 + i nu gamma_5) phi for a field whose last two axes are (spin, colour)."""
    return phi + 1j * nu * np.einsum("st,...tc->...sc", gamma5(), phi)


def dirac_tm(phi, gauge, kappa, mu, phases, dagger=False):
    """Twisted-mass operator D_tm = 1 + 2 i kappa mu gamma_5 - kappa H (D_tm^+: -mu and H^+), full lattice."""
    nu = (-2.0 if dagger else 2.0) * kappa * mu
    return twist(phi, nu) - kappa * hop(phi, gauge, phases, dagger)


def schur_tm(phi_e, gauge, kappa, mu, phases, dagger=False):
    """D_hat_tm phi_e = A phi_e - kappa^2 H_eo A^-1 H_oe phi_e, A = 1 + 2 i kappa mu gamma_5 (A^+ for the dagger)."""
    nu = (-2.0 if dagger else 2.0) * kappa * mu
    t = hop_eo(phi_e, 0, gauge, phases, dagger)
    t = twist(t, -nu) / (1.0 + nu * nu)
    return twist(phi_e, nu) - kappa * kappa * hop_eo(t, 1, gauge, phases, dagger)


def eo_prepare_tm(b_e, b_o, gauge, kappa, mu, phases):
    """bhat_e = b_e + kappa H_eo A^-1 b_o."""
    nu = 2.0 * kappa * mu
    return b_e + kappa * hop_eo(twist(b_o, -nu) / (1.0 + nu * nu), 1, gauge, phases)


def eo_reconstruct_tm(x_e, b_o, gauge, kappa, mu, phases):
    """x_o = A^-1 (b_o + kappa H_oe x_e)."""
    nu = 2.0 * kappa * mu
    return twist(b_o + kappa * hop_eo(x_e, 0, gauge, phases), -nu) / (1.0 + nu * nu)


def schur(phi_e, gauge, kappa, phases, dagger=False):
    """D_hat phi_e = phi_e - kappa^2 H_eo H_oe phi_e (D_hat^+ with H^+)."""
    t = hop_eo(phi_e, 0, gauge, phases, dagger)
    return phi_e - kappa * kappa * hop_eo(t, 1, gauge, phases, dagger)


def eo_prepare(b_e, b_o, gauge, kappa, phases):
    """Even-site source of the Schur system: b_hat = b_e + kappa H_eo b_o."""
    return b_e + kappa * hop_eo(b_o, 1, gauge, phases)


def eo_reconstruct(x_e, b_o, gauge, kappa, phases):
    """Odd-site solution from the even one: x_o = b_o + kappa H_oe x_e."""
    return b_o + kappa * hop_eo(x_e, 0, gauge, phases)


# --------------------------------------------------------------------------
# BLAS-1 and CG
# --------------------------------------------------------------------------
def dot(a, b) -> complex:
    """<a, b> = sum conj(a) b (FP64, numpy pairwise summation)."""
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return complex(np.sum(np.conj(a) * b))


def norm2(a) -> float:
    a = np.asarray(a).ravel()
    return float(np.sum(a.real * a.real + a.imag * a.imag))


def cg(apply_a, b, tol=1e-10, maxiter=10000, x0=None, fixed_iters=None,
       true_residual_restart=True):
    """Conjugate gradient (Hestenes-Stiefel) on a Hermitian positive definite A.

    Stops at the first iterate with ||r|| <= tol ||b|| on the iterated
    residual; then recomputes r = b - A x and, if that misses the tolerance,
    continues from the recomputed residual.  With ``fixed_iters`` set it runs
    exactly that many iterations and does no restart.

    Returns (x, info) with info = dict(iters, resid_history, true_rel_resid).
    """
    b = np.asarray(b, dtype=np.complex128)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.complex128)
    bnorm = np.sqrt(norm2(b))
    hist = []
    total = 0
    if bnorm == 0.0:
        return np.zeros_like(b), dict(iters=0, resid_history=[0.0], true_rel_resid=0.0)
    while True:
        r = b - apply_a(x) if (x0 is not None or total > 0) else b.copy()
        p = r.copy()
        rho = norm2(r)
        hist.append(np.sqrt(rho) / bnorm)
        while True:
            if fixed_iters is not None:
                if total >= fixed_iters:
                    break
            elif np.sqrt(rho) <= tol * bnorm or total >= maxiter:
                break
            q = apply_a(p)
            pq = dot(p, q).real
            alpha = rho / pq
            x = x + alpha * p
            r = r - alpha * q
            rho_new = norm2(r)
            beta = rho_new / rho
            p = r + beta * p
            rho = rho_new
            total += 1
            hist.append(np.sqrt(rho) / bnorm)
        true_rel = np.sqrt(norm2(b - apply_a(x))) / bnorm
        if (fixed_iters is not None or not true_residual_restart
                or true_rel <= tol or total >= maxiter):
            return x, dict(iters=total, resid_history=hist, true_rel_resid=true_rel)
        x0 = x


def cg_normal(apply_m, apply_mdag, b, **kw):
    """CG on the normal equations M^+ M x = b."""
    return cg(lambda v: apply_mdag(apply_m(v)), b, **kw)


# --------------------------------------------------------------------------
# Incremental EigCG (the paper's section on EigCG for twisted-mass fermions;
# algorithm of Stathopoulos and Orginos): CG on a Hermitian positive-definite
# A that also tracks a small search space of Lanczos vectors and keeps the
# lowest Ritz vectors; solutions of later right-hand sides start from the
# Galerkin projection onto the accumulated vectors (init-CG).
# --------------------------------------------------------------------------
class EigCG:
    """Plain restatement with numpy.  apply_a: A (Hermitian positive definite) on a flat complex vector."""

    def __init__(self, apply_a, nev=10, m=60, max_vectors=300):
        self.a, self.nev, self.m, self.max_vectors = apply_a, nev, m, max_vectors
        self.U = []          # orthonormal deflation vectors
        self.AU = []         # A applied to them
        self.ritz = []       # Rayleigh quotient u^+ A u of each kept vector

    def _init_guess(self, b):
        if not self.U:
            return np.zeros_like(b)
        U = np.stack(self.U, axis=1)
        H = U.conj().T @ np.stack(self.AU, axis=1)
        y = np.linalg.solve(H, U.conj().T @ b)
        return U @ y

    def solve(self, b, tol=1e-8, maxiter=100000, collect=True):
        """-> (x, iterations).  Collects nev Ritz vectors while the space has room."""
        b = np.asarray(b, dtype=np.complex128).ravel()
        x = self._init_guess(b)
        r = b - self.a(x)
        p = r.copy()
        rho = float(np.vdot(r, r).real)
        target = tol * tol * float(np.vdot(b, b).real)
        collect = collect and len(self.U) + self.nev <= self.max_vectors
        V, T = [], np.zeros((self.m, self.m))
        alpha_old = beta_old = None
        pending = None  # coupling row of the next basis vector after a restart
        k = it = 0
        while rho > target and it < maxiter:
            if collect:
                V.append(r / np.sqrt(rho))
                k = len(V)
            q = self.a(p)
            alpha = rho / float(np.vdot(p, q).real)
            x = x + alpha * p
            r = r - alpha * q
            rho_new = float(np.vdot(r, r).real)
            beta = rho_new / rho
            if collect:
                d = 1.0 / alpha + (beta_old / alpha_old if beta_old is not None else 0.0)
                T[k - 1, k - 1] = d
                if pending is not None:
                    T[: k - 1, k - 1] = pending
                    T[k - 1, : k - 1] = pending
                    pending = None
                off = -np.sqrt(beta) / alpha   # T_{k, k+1}: coupling to the next vector
                if k == self.m:
                    # restart: nev lowest Ritz vectors of T_m and of T_{m-1}
                    w, Y = np.linalg.eigh(T[:k, :k])
                    w1, Y1 = np.linalg.eigh(T[: k - 1, : k - 1])
                    Z = np.concatenate([Y[:, : self.nev], np.vstack([Y1[:, : self.nev], np.zeros((1, self.nev))])], axis=1)
                    Q, _ = np.linalg.qr(Z)
                    Vm = np.stack(V, axis=1) @ Q
                    V = [Vm[:, i] for i in range(Q.shape[1])]
                    Tn = Q.T @ T[:k, :k] @ Q
                    T = np.zeros((self.m, self.m))
                    T[: Q.shape[1], : Q.shape[1]] = Tn
                    pending = Q[k - 1, :] * off
                elif k < self.m:
                    T[k - 1, k] = T[k, k - 1] = off
            alpha_old, beta_old = alpha, beta
            p = r + beta * p
            rho = rho_new
            it += 1
        if collect and V:
            k = len(V)
            w, Y = np.linalg.eigh(T[:k, :k])
            W = np.stack(V, axis=1) @ Y[:, : self.nev]
            for i in range(W.shape[1]):
                v = W[:, i]
                for _ in range(2):
                    for u in self.U:
                        v = v - np.vdot(u, v) * u
                nv = np.linalg.norm(v)
                if nv < 1e-10:
                    continue
                v = v / nv
                self.U.append(v)
                self.AU.append(self.a(v))
                self.ritz.append(float(np.vdot(v, self.AU[-1]).real))
        return x, it


# --------------------------------------------------------------------------
# Link-spinor multiplication over a sequence of sites (the isolated kernel of
# the paper's addressing experiment, section on overlapping communication with
# computation): psi(x_i) = U(x_i) phi(x_i), U acting on the colour index of each
# of the four spin components.
# --------------------------------------------------------------------------
def su3_apply(u, phi, psi, sites):
    """u: (n, 3, 3), phi and psi: (n, 4, 3) complex; sites: site numbers x_i in step order.
    Returns a copy of psi with psi[x][s] = u[x] @ phi[x][s] for every spin s at each visited x;
    other sites keep their values."""
    out = np.array(psi, dtype=np.complex128, copy=True)
    for x in sites:
        for s in range(4):
            out[x, s] = u[x] @ phi[x, s]
    return out
