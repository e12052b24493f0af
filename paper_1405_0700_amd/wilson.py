"""Python binding of the Wilson-operator C ABI (``include/wilson.h``).

Argument marshalling only: every ``wl_*`` function below forwards to the
C function of the same name in ``libwilson.so``; all computation happens in
the library's HIP kernels.  Device buffers are passed as torch tensors (or raw
integer addresses) and the HIP stream defaults to torch's current stream.
There is no CPU fallback: if the library is missing, every call raises.
"""

from __future__ import annotations

import ctypes
import os
import re
from dataclasses import dataclass

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libwilson.so")
HEADER = os.path.join(os.path.dirname(_PKG), "include", "wilson.h")

# enums (wilson.h)
WL_OK, WL_NOT_CONVERGED, WL_BREAKDOWN = 0, 1, 2
WL_ERR_ARG, WL_ERR_DIMS, WL_ERR_HIP, WL_ERR_NOMEM, WL_ERR_UNSUPPORTED = -1, -2, -3, -4, -5
WL_F64, WL_F32, WL_F16N, WL_BF16N, WL_I16N = 0, 1, 2, 3, 4
WL_EVEN, WL_ODD, WL_FULL = 0, 1, 2
WL_OP_D, WL_OP_DHAT = 0, 1
WL_ACCESS_SEQ, WL_ACCESS_INDEX, WL_ACCESS_PTR = 0, 1, 2
WL_TCHUNK_AUTO = -1048576
WL_TCHUNK_YZ = -2097152

PREC = {"f64": WL_F64, "f32": WL_F32, "f16n": WL_F16N, "bf16n": WL_BF16N, "i16n": WL_I16N}
SUBSET = {"even": WL_EVEN, "odd": WL_ODD, "full": WL_FULL}
OP = {"D": WL_OP_D, "Dhat": WL_OP_DHAT}


class WilsonError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("wilson library error %d: %s" % (status, message))
        self.status = status


class SolverParams(ctypes.Structure):
    _fields_ = [
        ("tol", ctypes.c_double),
        ("maxiter", ctypes.c_int),
        ("check_every", ctypes.c_int),
        ("max_restarts", ctypes.c_int),
        ("prec", ctypes.c_int),
        ("recon", ctypes.c_int),
        ("reliable_every", ctypes.c_int),
        ("reliable_delta", ctypes.c_double),
        ("use_graph", ctypes.c_int),
        ("ru_restart", ctypes.c_int),
        ("mu", ctypes.c_double),
    ]


class SolverInfo(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int),
        ("restarts", ctypes.c_int),
        ("reliable_updates", ctypes.c_int),
        ("rel_resid", ctypes.c_double),
        ("true_rel_resid", ctypes.c_double),
        ("seconds", ctypes.c_double),
        ("fallback", ctypes.c_int),
        ("fallback_iters", ctypes.c_int),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class FgcrParams(ctypes.Structure):
    _fields_ = [
        ("tol", ctypes.c_double),
        ("maxiter", ctypes.c_int),
        ("restart", ctypes.c_int),
        ("fallback", ctypes.c_int),
        ("stagnation", ctypes.c_double),
    ]


class PcgnrParams(ctypes.Structure):
    _fields_ = [
        ("tol", ctypes.c_double),
        ("maxiter", ctypes.c_int),
        ("inner_tol", ctypes.c_double),
        ("fallback", ctypes.c_int),
        ("stagnation", ctypes.c_double),
    ]


_vp = ctypes.c_void_p
_ip = ctypes.POINTER(ctypes.c_int)
_dp = ctypes.POINTER(ctypes.c_double)
_SIGS = {
    "wl_ctx_create": (ctypes.c_int, [_ip, _dp, _dp, ctypes.POINTER(_vp)]),
    "wl_ctx_destroy": (ctypes.c_int, [_vp]),
    "wl_ctx_prepare_links": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int]),
    "wl_spinor_bytes": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)]),
    "wl_pack_spinor": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp]),
    "wl_unpack_spinor": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp]),
    "wl_convert_spinor": (ctypes.c_int, [_vp, _vp, ctypes.c_int, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp]),
    "wl_dslash_apply": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp]),
    "wl_dslash_dagger_apply": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp]),
    "wl_dirac_apply": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                      ctypes.c_int, ctypes.c_int, _vp]),
    "wl_eo_prepare": (ctypes.c_int, [_vp, _vp, _vp, _vp, ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp]),
    "wl_eo_reconstruct": (ctypes.c_int, [_vp, _vp, _vp, _vp, ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                         _vp]),
    "wl_blas_axpy": (ctypes.c_int, [_vp, ctypes.c_double, _vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp]),
    "wl_blas_dot": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp, _vp]),
    "wl_blas_norm2": (ctypes.c_int, [_vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp, _vp]),
    "wl_solver_params_default": (None, [ctypes.POINTER(SolverParams)]),
    "wl_cg_solve": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                   ctypes.POINTER(SolverParams), ctypes.POINTER(SolverInfo), _vp]),
    "wl_ctx_set_launch": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_void_p]),
    "wl_ctx_get_launch": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_void_p]),
    "wl_cgnr_solve": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_double, ctypes.c_int, ctypes.POINTER(SolverParams),
                                     ctypes.POINTER(SolverInfo), _vp]),
    "wl_fgcr_params_default": (None, [ctypes.POINTER(FgcrParams)]),
    "wl_pcgnr_params_default": (None, [ctypes.POINTER(PcgnrParams)]),
    "wl_eigcg_create": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_int, ctypes.POINTER(_vp)]),
    "wl_eigcg_destroy": (ctypes.c_int, [_vp]),
    "wl_eigcg_solve": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                      ctypes.POINTER(SolverInfo), _vp]),
    "wl_eigcg_vectors": (ctypes.c_int, [_vp, _ip, _dp]),
    "wl_eigcg_eigenvalues": (ctypes.c_int, [_vp, _ip, _dp]),
    "wl_su3_apply": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_long, ctypes.c_int, ctypes.c_int, _vp, _vp, _vp]),
    "wl_dslash_apply_split": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                             _vp]),
    "wl_dirac_tm_apply": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp]),
    "wl_eo_prepare_tm": (ctypes.c_int, [_vp, _vp, _vp, _vp, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                        ctypes.c_int, ctypes.c_int, _vp]),
    "wl_eo_reconstruct_tm": (ctypes.c_int, [_vp, _vp, _vp, _vp, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                            ctypes.c_int, ctypes.c_int, _vp]),
    "wl_batch_create": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int, ctypes.POINTER(_vp)]),
    "wl_batch_destroy": (ctypes.c_int, [_vp]),
    "wl_batch_set_launch": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    "wl_batch_get_launch": (ctypes.c_int, [_vp, _ip, _ip, _ip, _ip]),
    "wl_batch_dirac_apply": (ctypes.c_int, [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.c_int, ctypes.c_int,
                                            _dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp]),
    "wl_batch_cg_solve": (ctypes.c_int, [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.c_int, _dp, ctypes.c_int,
                                         ctypes.POINTER(SolverParams), ctypes.POINTER(SolverInfo), _vp]),
    "wl_batch_timing_enable": (ctypes.c_int, [_vp, ctypes.c_int]),
    "wl_autotune": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_char_p, _vp, _dp, _ip]),
    "wl_batch_autotune": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_char_p, _ip, _ip, _ip,
                                         _ip, _dp, _ip]),
    "wl_batch_timing_read": (ctypes.c_int, [_vp, _ip, _dp]),
    "wl_pcgnr_solve": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_double, _vp, ctypes.c_int,
                                      ctypes.POINTER(PcgnrParams), ctypes.POINTER(SolverInfo), _vp]),
    "wl_fgcr_solve": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_double, _vp, ctypes.POINTER(FgcrParams),
                                     ctypes.POINTER(SolverInfo), _vp]),
    "wl_ptc_create": (ctypes.c_int, [ctypes.c_int, _dp, _dp, ctypes.POINTER(_vp)]),
    "wl_ptc_destroy": (ctypes.c_int, [_vp]),
    "wl_ptc_get_weights": (ctypes.c_int, [_vp, _dp, _dp]),
    "wl_ptc_get_grads": (ctypes.c_int, [_vp, _dp, _dp]),
    "wl_ptc_get_moments": (ctypes.c_int, [_vp, _dp, _dp, _dp, _dp]),
    "wl_blas_dot_noalloc": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp, _vp]),
    "wl_ptc_apply": (ctypes.c_int, [_vp, _vp, _vp, _vp, ctypes.c_int, ctypes.c_int, _vp]),
    "wl_ptc_layer": (ctypes.c_int, [_vp, _vp, _vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp]),
    "wl_ptc_weight_grad": (ctypes.c_int, [_vp, _vp, _vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp]),
    "wl_ptc_accumulate": (ctypes.c_int, [_vp, _vp, _vp, _vp, ctypes.c_double, _vp]),
    "wl_ptc_accumulate_residual": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_double, ctypes.c_double, _vp]),
    "wl_ptc_step": (ctypes.c_int, [_vp, ctypes.c_double, _dp, _vp]),
    "wl_timing_enable": (ctypes.c_int, [_vp, ctypes.c_int]),
    "wl_timing_read": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _ip, _dp]),
    "wl_last_error": (ctypes.c_char_p, []),
    "wl_version": (ctypes.c_char_p, []),
}

_lib = None


def header_functions(path: str = HEADER):
    """Names of every function declared in include/wilson.h."""
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(wl_[a-z0-9_]+)\s*\(", text)))


def lib():
    """Load libwilson.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libwilson.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
        # torch ships its own HIP runtime; importing it first makes libwilson bind
        # to that same runtime instead of mapping a second one into the process
        import torch  # noqa: F401
        l = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(l, name)
            f.restype = res
            f.argtypes = args
        _lib = l
    return _lib


def last_error() -> str:
    return lib().wl_last_error().decode()


def _check(status):
    if status < 0:
        raise WilsonError(status, last_error())
    return status


def _ptr(x):
    """Device address of a field argument: a raw int is passed through, a torch
    tensor must live on the GPU and be contiguous (a host address or a strided
    view would be read by the kernels as device memory of the documented layout)."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if not getattr(x, "is_cuda", False):
        raise ValueError("field arguments must be device tensors (got %s)" % getattr(x, "device", type(x).__name__))
    if not x.is_contiguous():
        raise ValueError("field arguments must be contiguous tensors")
    return x.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


# ---------------------------------------------------------------- 1:1 wrappers
def wl_ctx_create(dims, phases, gauge_host: np.ndarray) -> int:
    g = np.ascontiguousarray(gauge_host, dtype=np.complex128)
    d = (ctypes.c_int * 4)(*[int(v) for v in dims])
    z = np.asarray(phases, dtype=np.complex128).reshape(4)
    ph = np.ascontiguousarray(np.stack([z.real, z.imag], -1).reshape(8))
    out = _vp()
    _check(lib().wl_ctx_create(d, ph.ctypes.data_as(_dp), g.view(np.float64).ctypes.data_as(_dp), ctypes.byref(out)))
    return out.value


def wl_ctx_destroy(ctx):
    return _check(lib().wl_ctx_destroy(ctx))


def wl_ctx_prepare_links(ctx, prec, recon):
    return _check(lib().wl_ctx_prepare_links(ctx, prec, recon))


def wl_spinor_bytes(ctx, subset, prec, nrhs=1) -> int:
    n = ctypes.c_size_t()
    _check(lib().wl_spinor_bytes(ctx, subset, prec, nrhs, ctypes.byref(n)))
    return n.value


def wl_pack_spinor(ctx, dst, src, subset, prec, nrhs=1, stream=None):
    return _check(lib().wl_pack_spinor(ctx, _ptr(dst), _ptr(src), subset, prec, nrhs, _stream(stream)))


def wl_unpack_spinor(ctx, dst, src, subset, prec, nrhs=1, stream=None):
    return _check(lib().wl_unpack_spinor(ctx, _ptr(dst), _ptr(src), subset, prec, nrhs, _stream(stream)))


def wl_convert_spinor(ctx, dst, dprec, src, sprec, subset, nrhs=1, stream=None):
    return _check(lib().wl_convert_spinor(ctx, _ptr(dst), dprec, _ptr(src), sprec, subset, nrhs, _stream(stream)))


def wl_dslash_apply(ctx, out, inp, subset, prec=WL_F64, recon=18, nrhs=1, stream=None):
    return _check(lib().wl_dslash_apply(ctx, _ptr(out), _ptr(inp), subset, prec, recon, nrhs, _stream(stream)))


def wl_dslash_dagger_apply(ctx, out, inp, subset, prec=WL_F64, recon=18, nrhs=1, stream=None):
    return _check(lib().wl_dslash_dagger_apply(ctx, _ptr(out), _ptr(inp), subset, prec, recon, nrhs,
                                               _stream(stream)))


def wl_dirac_apply(ctx, out, inp, op, dagger, kappa, prec=WL_F64, recon=18, nrhs=1, stream=None):
    return _check(lib().wl_dirac_apply(ctx, _ptr(out), _ptr(inp), op, int(bool(dagger)), float(kappa), prec, recon,
                                       nrhs, _stream(stream)))


def wl_eo_prepare(ctx, bhat_e, b_e, b_o, kappa, prec=WL_F64, recon=18, nrhs=1, stream=None):
    return _check(lib().wl_eo_prepare(ctx, _ptr(bhat_e), _ptr(b_e), _ptr(b_o), float(kappa), prec, recon, nrhs,
                                      _stream(stream)))


def wl_eo_reconstruct(ctx, x_o, x_e, b_o, kappa, prec=WL_F64, recon=18, nrhs=1, stream=None):
    return _check(lib().wl_eo_reconstruct(ctx, _ptr(x_o), _ptr(x_e), _ptr(b_o), float(kappa), prec, recon, nrhs,
                                          _stream(stream)))


def wl_blas_axpy(ctx, a, x, y, subset, prec=WL_F64, nrhs=1, stream=None):
    return _check(lib().wl_blas_axpy(ctx, float(a), _ptr(x), _ptr(y), subset, prec, nrhs, _stream(stream)))


def wl_blas_dot(ctx, x, y, subset, prec=WL_F64, nrhs=1, stream=None) -> complex:
    out = (ctypes.c_double * 2)()
    _check(lib().wl_blas_dot(ctx, _ptr(x), _ptr(y), subset, prec, nrhs, out, _stream(stream)))
    return complex(out[0], out[1])


def wl_blas_dot_noalloc(ctx, x, y, subset, prec=WL_F64, nrhs=1, result=None, stream=None):
    """<x, y> summed over rhs into the device tensor `result` (2 float64: re, im); asynchronous, no allocation
    inside the library (the static-scratch variant of wl_blas_dot)."""
    return _check(lib().wl_blas_dot_noalloc(ctx, _ptr(x), _ptr(y), subset, prec, nrhs, _ptr(result), _stream(stream)))


def wl_blas_norm2(ctx, x, subset, prec=WL_F64, nrhs=1, stream=None) -> float:
    out = ctypes.c_double()
    _check(lib().wl_blas_norm2(ctx, _ptr(x), subset, prec, nrhs, ctypes.byref(out), _stream(stream)))
    return out.value


def wl_solver_params_default() -> SolverParams:
    p = SolverParams()
    lib().wl_solver_params_default(ctypes.byref(p))
    return p


def wl_cg_solve(ctx, x, b, op, kappa, nrhs=1, params: SolverParams | None = None, stream=None):
    """Returns (status, [info dict per rhs]); raises on negative status."""
    p = params if params is not None else wl_solver_params_default()
    info = (SolverInfo * nrhs)()
    st = _check(lib().wl_cg_solve(ctx, _ptr(x), _ptr(b), op, float(kappa), nrhs, ctypes.byref(p), info,
                                  _stream(stream)))
    return st, [info[i].as_dict() for i in range(nrhs)]


class Launch(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int), ("swizzle", ctypes.c_int), ("tps", ctypes.c_int), ("tchunk", ctypes.c_int),
                ("nt", ctypes.c_int), ("rpt", ctypes.c_int), ("occ", ctypes.c_int), ("sweep", ctypes.c_int)]

    def as_tuple(self):
        return (self.block, self.swizzle, self.tps, self.tchunk, self.nt, self.rpt, self.occ, self.sweep)


def wl_cgnr_solve(ctx, x, eta, kappa, params: SolverParams | None = None, stream=None, nrhs=1):
    """Plain FP64 CG for D x = eta stopped on ||eta - D x|| <= tol ||eta||.
    Returns (status, info dict), or (status, [info dict per rhs]) for nrhs > 1."""
    p = params if params is not None else wl_solver_params_default()
    info = (SolverInfo * nrhs)()
    st = _check(lib().wl_cgnr_solve(ctx, _ptr(x), _ptr(eta), float(kappa), int(nrhs), ctypes.byref(p), info,
                                    _stream(stream)))
    out = [info[i].as_dict() for i in range(nrhs)]
    return st, (out[0] if nrhs == 1 else out)


def wl_fgcr_params_default() -> FgcrParams:
    p = FgcrParams()
    lib().wl_fgcr_params_default(ctypes.byref(p))
    return p


def wl_fgcr_solve(ctx, x, b, kappa, net=None, params: FgcrParams | None = None, stream=None):
    """FGCR on D x = b preconditioned by the PTC network `net` (None: no preconditioner)."""
    p = params if params is not None else wl_fgcr_params_default()
    info = SolverInfo()
    st = _check(lib().wl_fgcr_solve(ctx, _ptr(x), _ptr(b), float(kappa), net, ctypes.byref(p), ctypes.byref(info),
                                    _stream(stream)))
    return st, info.as_dict()


def wl_dirac_tm_apply(ctx, out, inp, op, dagger, kappa, mu, prec=WL_F64, recon=18, nrhs=1, stream=None):
    return _check(lib().wl_dirac_tm_apply(ctx, _ptr(out), _ptr(inp), op, int(bool(dagger)), float(kappa), float(mu),
                                          prec, recon, nrhs, _stream(stream)))


def wl_eo_prepare_tm(ctx, bhat_e, b_e, b_o, kappa, mu, prec=WL_F64, recon=18, nrhs=1, stream=None):
    return _check(lib().wl_eo_prepare_tm(ctx, _ptr(bhat_e), _ptr(b_e), _ptr(b_o), float(kappa), float(mu), prec, recon,
                                         nrhs, _stream(stream)))


def wl_eo_reconstruct_tm(ctx, x_o, x_e, b_o, kappa, mu, prec=WL_F64, recon=18, nrhs=1, stream=None):
    return _check(lib().wl_eo_reconstruct_tm(ctx, _ptr(x_o), _ptr(x_e), _ptr(b_o), float(kappa), float(mu), prec,
                                             recon, nrhs, _stream(stream)))


def wl_eigcg_create(ctx, op, kappa, mu=0.0, nev=10, m=60, max_vectors=300):
    out = _vp()
    _check(lib().wl_eigcg_create(ctx, int(op), float(kappa), float(mu), int(nev), int(m), int(max_vectors),
                                 ctypes.byref(out)))
    return out.value


def wl_eigcg_destroy(e):
    return _check(lib().wl_eigcg_destroy(e))


def wl_eigcg_solve(e, x, b, tol=1e-8, maxiter=100000, collect=True, stream=None):
    info = SolverInfo()
    st = _check(lib().wl_eigcg_solve(e, _ptr(x), _ptr(b), float(tol), int(maxiter), int(bool(collect)),
                                     ctypes.byref(info), _stream(stream)))
    return st, info.as_dict()


def wl_eigcg_vectors(e, max_vectors=300):
    n = ctypes.c_int()
    buf = (ctypes.c_double * max(1, max_vectors))()
    _check(lib().wl_eigcg_vectors(e, ctypes.byref(n), buf))
    return list(buf[: n.value])


def wl_eigcg_eigenvalues(e, max_vectors=300):
    """Eigenvalues of H = U^+ A U (the Ritz values on the whole deflation space), ascending."""
    n = ctypes.c_int()
    buf = (ctypes.c_double * max(1, max_vectors))()
    _check(lib().wl_eigcg_eigenvalues(e, ctypes.byref(n), buf))
    return list(buf[: n.value])


def wl_su3_apply(psi, u, phi, n, mode=WL_ACCESS_SEQ, layout=0, index=None, ptrs=None, stream=None):
    """psi(x_i) = U(x_i) phi(x_i) for i < n (device tensors; see wilson.h for modes and layouts)."""
    return _check(lib().wl_su3_apply(_ptr(psi), _ptr(u), _ptr(phi), int(n), int(mode), int(layout), _ptr(index),
                                     _ptr(ptrs), _stream(stream)))


def wl_dslash_apply_split(ctx, out, inp, subset, prec=WL_F64, recon=18, dagger=False, stream=None):
    """H in (H^+ in) for one output parity, bulk / boundary split with t-face exchange."""
    return _check(lib().wl_dslash_apply_split(ctx, _ptr(out), _ptr(inp), int(subset), int(prec), int(recon),
                                              int(bool(dagger)), _stream(stream)))


def _ptr_array(items):
    return (_vp * len(items))(*[_ptr(t) for t in items])


def wl_batch_create(ctxs):
    arr = (_vp * len(ctxs))(*ctxs)
    out = _vp()
    _check(lib().wl_batch_create(arr, len(ctxs), ctypes.byref(out)))
    return out.value


def wl_batch_destroy(batch):
    return _check(lib().wl_batch_destroy(batch))


def wl_batch_set_launch(batch, workgroups, block=256, nt=-1, tps=1):
    return _check(lib().wl_batch_set_launch(batch, int(workgroups), int(block), int(nt), int(tps)))


def wl_batch_get_launch(batch):
    """-> (workgroups, block, nt, tps)"""
    w, b, n, t = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check(lib().wl_batch_get_launch(batch, ctypes.byref(w), ctypes.byref(b), ctypes.byref(n), ctypes.byref(t)))
    return w.value, b.value, n.value, t.value


def wl_batch_dirac_apply(batch, outs, ins, op, dagger, kappas, prec=WL_F64, recon=18, nrhs=1, stream=None):
    k = (ctypes.c_double * len(kappas))(*[float(v) for v in kappas])
    return _check(lib().wl_batch_dirac_apply(batch, _ptr_array(outs), _ptr_array(ins), int(op), int(bool(dagger)), k,
                                             int(prec), int(recon), int(nrhs), _stream(stream)))


def wl_batch_cg_solve(batch, xs, bs, op, kappas, nrhs=1, params: SolverParams | None = None, stream=None):
    """Returns (status, [[info per rhs] per system])."""
    p = params if params is not None else wl_solver_params_default()
    n = len(xs)
    k = (ctypes.c_double * n)(*[float(v) for v in kappas])
    info = (SolverInfo * (n * nrhs))()
    st = _check(lib().wl_batch_cg_solve(batch, _ptr_array(xs), _ptr_array(bs), int(op), k, int(nrhs),
                                        ctypes.byref(p), info, _stream(stream)))
    return st, [[info[s * nrhs + r].as_dict() for r in range(nrhs)] for s in range(n)]


def wl_batch_timing_enable(batch, enable=True):
    return _check(lib().wl_batch_timing_enable(batch, int(bool(enable))))


def wl_batch_timing_read(batch):
    n, ms = ctypes.c_int(), ctypes.c_double()
    _check(lib().wl_batch_timing_read(batch, ctypes.byref(n), ctypes.byref(ms)))
    return n.value, ms.value


def wl_autotune(ctx, prec=WL_F64, recon=18, nrhs=1, cache_path=None):
    """Sweep the hopping-kernel launch shapes; returns (Launch tuple, microseconds per launch, from_cache)."""
    cfg = Launch()
    us = ctypes.c_double()
    fc = ctypes.c_int()
    path = None if cache_path is None else str(cache_path).encode()
    _check(lib().wl_autotune(ctx, int(prec), int(recon), int(nrhs), path, ctypes.addressof(cfg), ctypes.byref(us),
                             ctypes.byref(fc)))
    return cfg.as_tuple(), us.value, bool(fc.value)


def wl_batch_autotune(batch, prec=WL_F32, recon=18, nrhs=1, cache_path=None):
    """Sweep persistent workgroups / tile size / non-temporal hints / threads per point;
    returns ((workgroups, block, nt, tps), us, from_cache)."""
    w, b, n, t, fc = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    us = ctypes.c_double()
    path = None if cache_path is None else str(cache_path).encode()
    _check(lib().wl_batch_autotune(batch, int(prec), int(recon), int(nrhs), path, ctypes.byref(w), ctypes.byref(b),
                                   ctypes.byref(n), ctypes.byref(t), ctypes.byref(us), ctypes.byref(fc)))
    return (w.value, b.value, n.value, t.value), us.value, bool(fc.value)


def wl_pcgnr_params_default() -> PcgnrParams:
    p = PcgnrParams()
    lib().wl_pcgnr_params_default(ctypes.byref(p))
    return p


def wl_pcgnr_solve(ctx, x, b, kappa, net=None, params: PcgnrParams | None = None, stream=None, nrhs=1):
    """CG on the normal equations of D M y = b, x = M y, M the PTC network `net` (None: M = 1), for nrhs
    right-hand sides.  Returns (status, info dict), or (status, [info dict per rhs]) for nrhs > 1."""
    p = params if params is not None else wl_pcgnr_params_default()
    info = (SolverInfo * nrhs)()
    st = _check(lib().wl_pcgnr_solve(ctx, _ptr(x), _ptr(b), float(kappa), net, int(nrhs), ctypes.byref(p), info,
                                     _stream(stream)))
    out = [info[i].as_dict() for i in range(nrhs)]
    return st, (out[0] if nrhs == 1 else out)


def _cplx_flat(w):
    a = np.ascontiguousarray(np.asarray(w, dtype=np.complex128))
    return a, a.view(np.float64).ctypes.data_as(_dp)


def wl_ptc_create(w1, w2) -> int:
    """w1: (9, C, 1, 4, 4), w2: (9, 1, C, 4, 4) complex host arrays."""
    a1, p1 = _cplx_flat(w1)
    a2, p2 = _cplx_flat(w2)
    assert a1.shape[0] == 9 and a1.shape[2] == 1 and a2.shape[1] == 1 and a2.shape[2] == a1.shape[1]
    out = _vp()
    _check(lib().wl_ptc_create(int(a1.shape[1]), p1, p2, ctypes.byref(out)))
    return out.value


def wl_ptc_destroy(net):
    return _check(lib().wl_ptc_destroy(net))


def _ptc_pair(fn, net, channels):
    a = np.zeros((9, channels, 1, 4, 4), dtype=np.complex128)
    b = np.zeros((9, 1, channels, 4, 4), dtype=np.complex128)
    _check(fn(net, a.view(np.float64).ctypes.data_as(_dp), b.view(np.float64).ctypes.data_as(_dp)))
    return a, b


def wl_ptc_get_weights(net, channels):
    return _ptc_pair(lib().wl_ptc_get_weights, net, channels)


def wl_ptc_get_grads(net, channels):
    return _ptc_pair(lib().wl_ptc_get_grads, net, channels)


def wl_ptc_get_moments(net, channels):
    """-> (m1, m2, v1, v2): Adam's moments of (Re W, Im W), shapes w.shape + (2,) (float64)."""
    m1 = np.zeros((9, channels, 1, 4, 4, 2))
    m2 = np.zeros((9, 1, channels, 4, 4, 2))
    v1, v2 = np.zeros_like(m1), np.zeros_like(m2)
    _check(lib().wl_ptc_get_moments(net, *(a.ctypes.data_as(_dp) for a in (m1, m2, v1, v2))))
    return m1, m2, v1, v2


def wl_ptc_apply(ctx, net, out, inp, stream=None, nrhs=1, adjoint=False):
    return _check(lib().wl_ptc_apply(ctx, net, _ptr(out), _ptr(inp), int(nrhs), int(bool(adjoint)), _stream(stream)))


def wl_ptc_layer(ctx, out, inp, weights, cout, cin, adjoint=False, stream=None):
    return _check(lib().wl_ptc_layer(ctx, _ptr(out), _ptr(inp), _ptr(weights), int(cout), int(cin),
                                     int(bool(adjoint)), _stream(stream)))


def wl_ptc_weight_grad(ctx, grad, g_out, inp, cout, cin, accumulate=False, stream=None):
    return _check(lib().wl_ptc_weight_grad(ctx, _ptr(grad), _ptr(g_out), _ptr(inp), int(cout), int(cin),
                                           int(bool(accumulate)), _stream(stream)))


def wl_ptc_accumulate(ctx, net, r, e, inv_npairs, stream=None):
    return _check(lib().wl_ptc_accumulate(ctx, net, _ptr(r), _ptr(e), float(inv_npairs), _stream(stream)))


def wl_ptc_accumulate_residual(ctx, net, r, kappa, inv_npairs, stream=None):
    return _check(lib().wl_ptc_accumulate_residual(ctx, net, _ptr(r), float(kappa), float(inv_npairs),
                                                   _stream(stream)))


def wl_ptc_step(net, lr, stream=None) -> float:
    loss = ctypes.c_double()
    _check(lib().wl_ptc_step(net, float(lr), ctypes.byref(loss), _stream(stream)))
    return loss.value


def wl_ctx_set_launch(ctx, prec, block, swizzle, tps, tchunk=WL_TCHUNK_AUTO, nt=-1, rpt=1, occ=0, sweep=0):
    cfg = Launch(int(block), int(swizzle), int(tps), int(tchunk), int(nt), int(rpt), int(occ), int(sweep))
    return _check(lib().wl_ctx_set_launch(ctx, prec, ctypes.addressof(cfg)))


def wl_ctx_get_launch(ctx, prec):
    """-> (block, swizzle, tps, tchunk, nt, rpt, occ, sweep)"""
    cfg = Launch()
    _check(lib().wl_ctx_get_launch(ctx, prec, ctypes.addressof(cfg)))
    return cfg.as_tuple()


def wl_timing_enable(ctx, enable=True, every=1):
    """Record every `every`-th hopping launch (enable=False: stop)."""
    return _check(lib().wl_timing_enable(ctx, int(every) if enable else 0))


def wl_timing_read(ctx, prec, recon, dagger, epilogue):
    """-> (count, total_ms) of the recorded hopping-kernel launches of that variant."""
    n = ctypes.c_int()
    ms = ctypes.c_double()
    _check(lib().wl_timing_read(ctx, prec, recon, int(bool(dagger)), epilogue, ctypes.byref(n), ctypes.byref(ms)))
    return n.value, ms.value


def wl_version() -> str:
    return lib().wl_version().decode()


# ---------------------------------------------------------------- convenience
@dataclass
class Lattice:
    """A context plus helpers that allocate internal fields as torch tensors."""

    dims: tuple
    phases: tuple
    ctx: int

    @classmethod
    def create(cls, gauge: np.ndarray, phases=(1, 1, 1, -1)):
        lt, lz, ly, lx = gauge.shape[:4]
        dims = (lx, ly, lz, lt)
        return cls(dims, tuple(complex(p) for p in phases), wl_ctx_create(dims, phases, gauge))

    def close(self):
        if self.ctx:
            wl_ctx_destroy(self.ctx)
            self.ctx = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def volume(self):
        return int(np.prod(self.dims))

    def new(self, subset=WL_FULL, prec=WL_F64, nrhs=1, zero=True):
        import torch
        n = wl_spinor_bytes(self.ctx, subset, prec, nrhs)
        f = torch.empty(n, dtype=torch.uint8, device="cuda")
        if zero:
            f.zero_()
        return f

    def pack(self, canonical, subset=WL_FULL, prec=WL_F64, nrhs=1):
        """canonical numpy/torch complex128 field -> new internal field."""
        import torch
        t = torch.as_tensor(np.ascontiguousarray(canonical)) if isinstance(canonical, np.ndarray) else canonical
        t = t.to(device="cuda", dtype=torch.complex128).contiguous()
        out = self.new(subset, prec, nrhs, zero=False)
        wl_pack_spinor(self.ctx, out, t, subset, prec, nrhs)
        return out

    def unpack(self, internal, subset=WL_FULL, prec=WL_F64, nrhs=1) -> np.ndarray:
        """internal field -> numpy complex128, shape (nrhs, nsites, 4, 3) (nrhs axis dropped if 1)."""
        import torch
        nsite = self.volume if subset == WL_FULL else self.volume // 2
        out = torch.empty((nrhs, nsite, 4, 3), dtype=torch.complex128, device="cuda")
        wl_unpack_spinor(self.ctx, out, internal, subset, prec, nrhs)
        torch.cuda.synchronize()
        a = out.cpu().numpy()
        return a[0] if nrhs == 1 else a
