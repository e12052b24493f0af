"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function that include/wilson.h declares, and rejects bad arguments with
the documented status codes before touching the device."""

import ctypes

import numpy as np
import pytest

from paper_1405_0700_amd import wilson as W


@pytest.fixture(scope="module")
def lib():
    return W.lib()


def test_exports_every_header_function(lib):
    names = W.header_functions()
    assert len(names) >= 18
    for n in names:
        assert hasattr(lib, n), n
        assert n in W._SIGS, "binding lacks " + n


def test_version_and_defaults(lib):
    assert W.wl_version().startswith("wilson-gfx950")
    p = W.wl_solver_params_default()
    assert p.tol == 1e-10 and p.maxiter == 100000 and p.prec == W.WL_F64 and p.recon == 18
    assert p.check_every == 25 and p.reliable_every == 100 and p.reliable_delta == 0.1
    assert p.use_graph == 0 and p.ru_restart == -1


def _create(dims, phases=(1, 0, 1, 0, 1, 0, -1, 0), gauge=True):
    l = W.lib()
    d = (ctypes.c_int * 4)(*dims)
    ph = (ctypes.c_double * 8)(*phases)
    g = np.zeros(max(1, int(np.prod(dims))) * 72) if gauge else None
    gp = g.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if gauge else None
    out = ctypes.c_void_p()
    st = l.wl_ctx_create(d, ph, gp, ctypes.byref(out))
    return st, out


@pytest.mark.parametrize("dims", [(3, 4, 4, 4), (4, 4, 0, 4), (4, 4, 4, 5), (4, -2, 4, 4)])
def test_bad_extents_rejected(dims):
    st, out = _create(dims)
    assert st == W.WL_ERR_DIMS
    assert out.value is None
    assert "even" in W.last_error()


def test_null_arguments_rejected():
    st, _ = _create((4, 4, 4, 4), gauge=False)
    assert st == W.WL_ERR_ARG
    assert W.last_error()


def test_nonfinite_phase_rejected():
    st, _ = _create((4, 4, 4, 4), phases=(1, 0, float("nan"), 0, 1, 0, -1, 0))
    assert st == W.WL_ERR_ARG


def test_null_context_rejected(lib):
    n = ctypes.c_size_t()
    assert lib.wl_spinor_bytes(None, W.WL_FULL, W.WL_F64, 1, ctypes.byref(n)) == W.WL_ERR_ARG
    assert lib.wl_dslash_apply(None, 16, 32, W.WL_EVEN, W.WL_F64, 18, 1, None) == W.WL_ERR_ARG
    assert lib.wl_cg_solve(None, 16, 32, W.WL_OP_D, 0.1, 1, None, None, None) == W.WL_ERR_ARG
    assert lib.wl_ctx_destroy(None) == W.WL_OK


def test_no_device_is_an_error_not_a_crash():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    st, out = _create((4, 4, 4, 4))
    assert st == W.WL_ERR_HIP
    assert out.value is None
    assert "device" in W.last_error()


def test_binding_rejects_host_and_strided_tensors():
    # the binding checks field tensors before any library call: a host address or a
    # strided view would be read by the kernels as device memory of the field layout
    import torch
    host = torch.zeros(64, dtype=torch.uint8)
    with pytest.raises(ValueError, match="device"):
        W.wl_dslash_apply(None, host, host, W.WL_EVEN)
    with pytest.raises(ValueError, match="device"):
        W.wl_cg_solve(None, host, host, W.WL_OP_DHAT, 0.1)
    assert W._ptr(None) is None and W._ptr(4096) == 4096
