"""GPU parity of the HIP path against the FP64 CPU oracle, through the C ABI.

Tolerances (relative, normwise over the whole output field):
  FP64 storage      1e-13  (the operator sums 8 hops of ~100 rounded terms each;
                            observed differences are a few 1e-16)
  FP32 storage      2e-6   (inputs rounded to FP32, unit roundoff 6e-8, times
                            the ~30-term accumulation depth of one output)
  FP16 + site norm  4e-3   (unit roundoff 2^-11 = 4.9e-4 on inputs scaled by
                            the per-site maximum, same accumulation depth)
  BF16 + site norm  3e-2   (unit roundoff 2^-8 = 3.9e-3)
  int16 + site norm 3e-4   (fixed point: half a step of 2^-15 of the site maximum)
"""

import numpy as np
import pytest
import torch

from oracle import oracle as orc
from paper_1405_0700_amd import synth
from paper_1405_0700_amd import wilson as W

pytestmark = pytest.mark.gpu

TOL = {W.WL_F64: 1e-13, W.WL_F32: 2e-6, W.WL_F16N: 4e-3, W.WL_BF16N: 3e-2, W.WL_I16N: 3e-4}
AP = (1, 1, 1, -1)


@pytest.fixture(autouse=True)
def _announce(request):
    print("\n[gpu case] %s" % request.node.nodeid, flush=True)
    yield


def rel(a, b):
    return float(np.linalg.norm((np.asarray(a) - np.asarray(b)).ravel()) / np.linalg.norm(np.asarray(b).ravel()))


def random_phases(seed):
    rng = np.random.default_rng(seed)
    return tuple(np.exp(1j * rng.uniform(0, 2 * np.pi, 4)))


_cache = {}


def setup(dims, eps=0.5, seed=7, phases=AP):
    key = (dims, eps, seed, phases)
    if key not in _cache:
        u = synth.su3_links(dims, eps, seed)
        _cache[key] = (u, W.Lattice.create(u, phases))
    return _cache[key]


def full_shape(dims):
    lx, ly, lz, lt = dims
    return (lt, lz, ly, lx, 4, 3)


# ------------------------------------------------------------------ layout
@pytest.mark.parametrize("prec", [W.WL_F64, W.WL_F32])
@pytest.mark.parametrize("nrhs", [1, 3])
def test_pack_unpack_roundtrip(prec, nrhs):
    dims = (6, 4, 2, 4)
    _, lat = setup(dims)
    rng = np.random.default_rng(1)
    for subset, nsite in [(W.WL_FULL, 192), (W.WL_EVEN, 96), (W.WL_ODD, 96)]:
        f = rng.standard_normal((nrhs, nsite, 4, 3)) + 1j * rng.standard_normal((nrhs, nsite, 4, 3))
        if prec == W.WL_F32:
            f = f.astype(np.complex64).astype(np.complex128)
        back = lat.unpack(lat.pack(f, subset, prec, nrhs), subset, prec, nrhs)
        assert np.array_equal(back.reshape(f.shape), f)


def test_full_field_layout_is_even_then_odd():
    dims = (4, 6, 2, 4)
    _, lat = setup(dims)
    f = synth.gaussian_spinor(dims, seed=3)
    internal = lat.pack(f, W.WL_FULL)
    half = internal.numel() // 2
    e = lat.unpack(internal[:half], W.WL_EVEN)
    o = lat.unpack(internal[half:], W.WL_ODD)
    oe, oo = orc.eo_split(f, dims)
    assert np.array_equal(e, oe) and np.array_equal(o, oo)


@pytest.mark.parametrize("prec", [W.WL_F16N, W.WL_BF16N])
def test_half_storage_roundtrip_error(prec):
    dims = (4, 4, 4, 4)
    _, lat = setup(dims)
    f = synth.gaussian_spinor(dims, seed=5)
    f[0, 0, 0, 0] = 0  # an all-zero site must survive (norm 0 stores zeros)
    back = lat.unpack(lat.pack(f, W.WL_FULL, prec), W.WL_FULL, prec).reshape(f.shape)
    assert np.all(back[0, 0, 0, 0] == 0)
    u = 2.0 ** -11 if prec == W.WL_F16N else 2.0 ** -8
    # each component is off by at most half an ulp of the site maximum
    smax = np.max(np.maximum(np.abs(f.real), np.abs(f.imag)), axis=(-1, -2), keepdims=True)
    err = np.maximum(np.abs((back - f).real), np.abs((back - f).imag))
    assert np.all(err <= smax * u * 1.0001)


# ------------------------------------------------------------------ hopping term
CASES = [(8, 8, 8, 8), (6, 10, 4, 14), (2, 4, 2, 6)]


@pytest.mark.parametrize("dims", CASES)
@pytest.mark.parametrize("dagger", [False, True])
@pytest.mark.parametrize("recon", [18, 12])
def test_dslash_f64_all_subsets(dims, dagger, recon):
    ph = random_phases(11)
    u, lat = setup(dims, phases=ph)
    phi = synth.gaussian_spinor(dims, seed=12)
    want = orc.hop(phi, u, ph, dagger=dagger)
    we, wo = orc.eo_split(want, dims)
    pe, po = orc.eo_split(phi, dims)
    fn = W.wl_dslash_dagger_apply if dagger else W.wl_dslash_apply
    # full lattice
    out = lat.new(W.WL_FULL)
    fn(lat.ctx, out, lat.pack(phi), W.WL_FULL, W.WL_F64, recon)
    got = lat.unpack(out, W.WL_FULL).reshape(want.shape)
    assert rel(got, want) < TOL[W.WL_F64]
    # half lattices: out_e = H_eo in_o, out_o = H_oe in_e
    oe = lat.new(W.WL_EVEN)
    fn(lat.ctx, oe, lat.pack(po, W.WL_ODD), W.WL_EVEN, W.WL_F64, recon)
    assert rel(lat.unpack(oe, W.WL_EVEN), we) < TOL[W.WL_F64]
    oo = lat.new(W.WL_ODD)
    fn(lat.ctx, oo, lat.pack(pe, W.WL_EVEN), W.WL_ODD, W.WL_F64, recon)
    assert rel(lat.unpack(oo, W.WL_ODD), wo) < TOL[W.WL_F64]


@pytest.mark.parametrize("prec,recon", [(W.WL_F32, 18), (W.WL_F32, 12), (W.WL_F16N, 12), (W.WL_BF16N, 12),
                                        (W.WL_I16N, 12)])
@pytest.mark.parametrize("dagger", [False, True])
def test_dslash_low_precision(prec, recon, dagger):
    dims = (6, 10, 4, 14)
    u, lat = setup(dims)
    phi = synth.gaussian_spinor(dims, seed=21)
    want = orc.hop(phi, u, AP, dagger=dagger)
    out = lat.new(W.WL_FULL, prec)
    fn = W.wl_dslash_dagger_apply if dagger else W.wl_dslash_apply
    fn(lat.ctx, out, lat.pack(phi, W.WL_FULL, prec), W.WL_FULL, prec, recon)
    err = rel(lat.unpack(out, W.WL_FULL, prec).reshape(want.shape), want)
    print("prec", prec, "recon", recon, "rel err", err)
    assert err < TOL[prec]


def _quantize(x, prec):
    """The value a real FP64 link entry takes in the library's 16-bit link storage: FP16 is the FP64 value
    rounded once to nearest even (the conversion kernel converts FP64 -> FP32 -> FP16 in its source; the
    compiler merges the two into one FP64 -> FP16 rounding, done in integer arithmetic, and a twice-rounded
    reference differs from it in a few entries by one step); BF16 rounds the FP32 bit pattern, FP64 -> FP32
    -> BF16;
    int16 is round(32767 v) / 32767, decoded in FP32."""
    x32 = np.asarray(x, dtype=np.float32)
    if prec == W.WL_F16N:
        return np.asarray(x, dtype=np.float64).astype(np.float16).astype(np.float64)
    if prec == W.WL_BF16N:
        b = np.ascontiguousarray(x32).view(np.uint32).astype(np.uint64)
        b = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
        return b.astype(np.uint32).view(np.float32).astype(np.float64)
    q = np.clip(np.rint(x32 * np.float32(32767.0)), -32767, 32767).astype(np.float32)
    return (q * np.float32(1.0 / 32767.0)).astype(np.float64)


def _links_as_stored(u, prec):
    """12-real 16-bit links as the kernels see them: rows 0 and 1 quantized, row 2 = conj(row0 x row1)."""
    q = _quantize(u.real, prec) + 1j * _quantize(u.imag, prec)
    r0, r1 = q[..., 0, :], q[..., 1, :]
    r2 = np.conj(np.cross(r0, r1))
    return np.stack([r0, r1, r2], axis=-2)


@pytest.mark.parametrize("prec", [W.WL_F16N, W.WL_BF16N, W.WL_I16N])
@pytest.mark.parametrize("dagger", [False, True])
def test_dslash_16bit_per_site(prec, dagger):
    """Per-site check of the 16-bit formats (a normwise tolerance would let an error confined to a few
    sites pass): the oracle is fed the inputs exactly as stored (spinors unpacked from the 16-bit field,
    links quantized the same way with the third row rebuilt), so what remains at every site is the
    rounding of the output to its own per-point norm s_out (at most half a step of the format, relative
    to s_out) plus FP32 arithmetic (its a-priori bound, ARITH_F32 times the largest input component among
    the site's neighbours)."""
    dims = (6, 10, 4, 14)
    ph = random_phases(23)
    u, lat = setup(dims, seed=24, phases=ph)
    phi = synth.gaussian_spinor(dims, seed=25)
    # at some sites the input is scaled by 1e3 or 1e-3: the per-point norm must follow each site
    rng = np.random.default_rng(26)
    scale = rng.choice([1e-3, 1.0, 1e3], size=phi.shape[:4], p=[0.1, 0.8, 0.1])
    phi = phi * scale[..., None, None]
    inp = lat.pack(phi, W.WL_FULL, prec)
    phi_q = lat.unpack(inp, W.WL_FULL, prec).reshape(phi.shape)
    out = lat.new(W.WL_FULL, prec)
    (W.wl_dslash_dagger_apply if dagger else W.wl_dslash_apply)(lat.ctx, out, inp, W.WL_FULL, prec, 12)
    got = lat.unpack(out, W.WL_FULL, prec).reshape(phi.shape)
    want = orc.hop(phi_q, _links_as_stored(u, prec), ph, dagger=dagger)
    assert _per_site_worst(got, want, _neighbour_max(phi_q), prec, "dagger %d" % dagger) <= 1.0
    # and the normwise figure against the unquantized oracle stays within the format's tolerance
    assert rel(got, orc.hop(phi, u, ph, dagger=dagger)) < TOL[prec]


# Per-site bound of a 16-bit half-dslash output component: the rounding of the output to its per-point norm
# s_out (half a step of the format, relative to s_out), plus the FP32 arithmetic before it.  The latter is the
# a-priori bound of a rounded sum of products: unit roundoff 2^-24 times the accumulation depth (~30 sequential
# roundings per component) times the sum of the absolute terms, at most 8 hops x 3 colours x 2 real products
# x |U_ij| <= 1 x |h| <= 2 s_nb = 96 s_nb, s_nb the largest input component among the site's neighbours.
HALF_STEP = {W.WL_F16N: 2.0 ** -11, W.WL_BF16N: 2.0 ** -8, W.WL_I16N: 0.5 / 32767}
ARITH_F32 = 2.0 ** -24 * 30 * 96


def _comp(a):
    return np.maximum(np.abs(a.real), np.abs(a.imag)).max(axis=(-1, -2))


def _neighbour_max(phi_q):
    s_in = _comp(phi_q)
    s_nb = np.zeros_like(s_in)
    for axis in range(4):
        for sh in (1, -1):
            s_nb = np.maximum(s_nb, np.roll(s_in, sh, axis=axis))
    return s_nb


def _per_site_worst(got, want, s_nb, prec, label):
    """Largest per-site error over its bound; prints the worst site's error in units of each term."""
    err, s_out = _comp(got - want), _comp(want)
    ratio = err / (1.02 * HALF_STEP[prec] * s_out + ARITH_F32 * s_nb)
    k = np.unravel_index(np.argmax(ratio), ratio.shape)
    print("%s prec %d: worst per-site error / bound %.4f (error = %.3f rounding steps of s_out, %.2e s_nb)"
          % (label, prec, ratio[k], err[k] / (HALF_STEP[prec] * s_out[k]), err[k] / s_nb[k]))
    return float(ratio[k])


@pytest.mark.parametrize("prec", [W.WL_F16N, W.WL_BF16N])
def test_dslash_16bit_full_size_default_launch(prec):
    """FP16+norm and BF16+norm hopping term at 32^3x64 (the mixed-precision lattice, links exp(0.2 i H)
    seed 301, source seed 302) with the default launch: the full-lattice output (109 MB) is stored
    non-temporally, the even half-dslash the solvers launch (55 MB) through the caches.  Every site is
    checked against the oracle fed the inputs as stored, to the per-site bound of
    test_dslash_16bit_per_site.  Measured: the worst site of either format is half a step of its
    per-point norm, the output rounding alone (with a reference that rounded the FP16 links twice, through
    FP32, a few sites were one FP16 step further off: that is how the library's once-rounded FP16 links
    were found)."""
    dims = (32, 32, 32, 64)
    u, lat = setup(dims, eps=0.2, seed=301)
    phi = synth.gaussian_spinor(dims, seed=302)
    inp = lat.pack(phi, W.WL_FULL, prec)
    phi_q = lat.unpack(inp, W.WL_FULL, prec).reshape(phi.shape)
    want = orc.hop(phi_q, _links_as_stored(u, prec), AP)
    out = lat.new(W.WL_FULL, prec)
    W.wl_dslash_apply(lat.ctx, out, inp, W.WL_FULL, prec, 12)
    got = lat.unpack(out, W.WL_FULL, prec).reshape(phi.shape)
    s_nb = _neighbour_max(phi_q)
    assert _per_site_worst(got, want, s_nb, prec, "full lattice") <= 1.0
    # the even half-dslash from the odd half of the stored input
    _, po = orc.eo_split(phi_q, dims)
    oe = lat.new(W.WL_EVEN, prec)
    W.wl_dslash_apply(lat.ctx, oe, lat.pack(po, W.WL_ODD, prec), W.WL_EVEN, prec, 12)
    ge = lat.unpack(oe, W.WL_EVEN, prec)
    assert _per_site_worst(ge, orc.eo_split(want, dims)[0], orc.eo_split(s_nb, dims)[0], prec,
                           "even half-dslash") <= 1.0


def test_dslash_f64_headline_size_default_launch():
    """FP64 half-dslash and full hopping term at 24^3x48 (the headline lattice, links exp(0.2 i H) seed 201)
    with the default launch, which at this size uses the z-chunked order and non-temporal link loads; the
    half-dslash output (64 MB) is stored through the caches, the full one (128 MB) non-temporally.  Both store
    forms give the same bits as a launch without non-temporal hints."""
    dims = (24, 24, 24, 48)
    u = synth.su3_links(dims, 0.2, 201)
    lat = W.Lattice.create(u, AP)
    try:
        phi = synth.gaussian_spinor(dims, seed=202)
        want = orc.hop(phi, u, AP)
        we, wo = orc.eo_split(want, dims)
        pe, po = orc.eo_split(phi, dims)
        oe = lat.new(W.WL_EVEN)
        W.wl_dslash_apply(lat.ctx, oe, lat.pack(po, W.WL_ODD), W.WL_EVEN)
        assert rel(lat.unpack(oe, W.WL_EVEN), we) < TOL[W.WL_F64]
        od = lat.new(W.WL_ODD)
        W.wl_dslash_dagger_apply(lat.ctx, od, lat.pack(pe, W.WL_EVEN), W.WL_ODD)
        assert rel(lat.unpack(od, W.WL_ODD), orc.eo_split(orc.hop(phi, u, AP, dagger=True), dims)[1]) < TOL[W.WL_F64]
        out = lat.new(W.WL_FULL)
        W.wl_dslash_apply(lat.ctx, out, lat.pack(phi), W.WL_FULL)
        assert rel(lat.unpack(out).reshape(want.shape), want) < TOL[W.WL_F64]
        cfg = W.wl_ctx_get_launch(lat.ctx, W.WL_F64)
        block, swz, tps, tch, nt, rpt, occ, sweep = cfg
        W.wl_ctx_set_launch(lat.ctx, W.WL_F64, block, swz, tps, tch, 0, rpt, occ, sweep)
        oe0, out0 = lat.new(W.WL_EVEN), lat.new(W.WL_FULL)
        W.wl_dslash_apply(lat.ctx, oe0, lat.pack(po, W.WL_ODD), W.WL_EVEN)
        W.wl_dslash_apply(lat.ctx, out0, lat.pack(phi), W.WL_FULL)
        assert torch.equal(oe0, oe) and torch.equal(out0, out)
        W.wl_ctx_set_launch(lat.ctx, W.WL_F64, *cfg)
    finally:
        lat.close()


def test_dslash_multi_rhs_equals_single():
    dims = (6, 4, 4, 8)
    u, lat = setup(dims)
    n = 5
    fields = [synth.gaussian_spinor(dims, seed=100 + k) for k in range(n)]
    stack = np.stack([f.reshape(-1, 4, 3) for f in fields])
    for prec in (W.WL_F64, W.WL_F32):
        out = lat.new(W.WL_FULL, prec, n)
        W.wl_dslash_apply(lat.ctx, out, lat.pack(stack, W.WL_FULL, prec, n), W.WL_FULL, prec, 18, n)
        multi = lat.unpack(out, W.WL_FULL, prec, n)
        for k in range(n):
            o1 = lat.new(W.WL_FULL, prec)
            W.wl_dslash_apply(lat.ctx, o1, lat.pack(fields[k], W.WL_FULL, prec), W.WL_FULL, prec, 18)
            assert np.array_equal(multi[k], lat.unpack(o1, W.WL_FULL, prec))
        if prec == W.WL_F64:
            want = orc.hop(fields[2], u, AP)
            assert rel(multi[2].reshape(want.shape), want) < TOL[W.WL_F64]


def test_dslash_rejects_aliasing_and_bad_recon():
    dims = (4, 4, 4, 4)
    _, lat = setup(dims)
    f = lat.new(W.WL_FULL)
    with pytest.raises(W.WilsonError) as e:
        W.wl_dslash_apply(lat.ctx, f, f, W.WL_FULL)
    assert e.value.status == W.WL_ERR_ARG
    with pytest.raises(W.WilsonError) as e:
        W.wl_dslash_apply(lat.ctx, lat.new(W.WL_FULL, W.WL_F16N), lat.new(W.WL_FULL, W.WL_F16N), W.WL_FULL,
                          W.WL_F16N, 18)
    assert e.value.status == W.WL_ERR_UNSUPPORTED


# ------------------------------------------------------------------ Dirac operators
@pytest.mark.parametrize("dagger", [False, True])
def test_dirac_full_and_schur(dagger):
    dims = (6, 10, 4, 14)
    kappa = 0.135
    u, lat = setup(dims, eps=0.2, seed=9)
    phi = synth.gaussian_spinor(dims, seed=31)
    want = orc.dirac(phi, u, kappa, AP, dagger=dagger)
    out = lat.new(W.WL_FULL)
    W.wl_dirac_apply(lat.ctx, out, lat.pack(phi), W.WL_OP_D, dagger, kappa)
    assert rel(lat.unpack(out).reshape(want.shape), want) < TOL[W.WL_F64]
    pe, _ = orc.eo_split(phi, dims)
    want_e = orc.schur(pe, u, kappa, AP, dagger=dagger)
    oe = lat.new(W.WL_EVEN)
    W.wl_dirac_apply(lat.ctx, oe, lat.pack(pe, W.WL_EVEN), W.WL_OP_DHAT, dagger, kappa)
    assert rel(lat.unpack(oe, W.WL_EVEN), want_e) < TOL[W.WL_F64]


def test_eo_prepare_and_reconstruct():
    dims = (6, 4, 4, 8)
    kappa = 0.12
    u, lat = setup(dims)
    b = synth.gaussian_spinor(dims, seed=41)
    x = synth.gaussian_spinor(dims, seed=42)
    be, bo = orc.eo_split(b, dims)
    xe, _ = orc.eo_split(x, dims)
    bh = lat.new(W.WL_EVEN)
    W.wl_eo_prepare(lat.ctx, bh, lat.pack(be, W.WL_EVEN), lat.pack(bo, W.WL_ODD), kappa)
    assert rel(lat.unpack(bh, W.WL_EVEN), orc.eo_prepare(be, bo, u, kappa, AP)) < TOL[W.WL_F64]
    xo = lat.new(W.WL_ODD)
    W.wl_eo_reconstruct(lat.ctx, xo, lat.pack(xe, W.WL_EVEN), lat.pack(bo, W.WL_ODD), kappa)
    assert rel(lat.unpack(xo, W.WL_ODD), orc.eo_reconstruct(xe, bo, u, kappa, AP)) < TOL[W.WL_F64]


# ------------------------------------------------------------------ BLAS
def test_blas_exact_on_integer_data():
    dims = (6, 10, 4, 14)
    _, lat = setup(dims)
    rng = np.random.default_rng(3)
    shp = full_shape(dims)
    x = rng.integers(-8, 9, shp) + 1j * rng.integers(-8, 9, shp)
    y = rng.integers(-8, 9, shp) + 1j * rng.integers(-8, 9, shp)
    X, Y = lat.pack(x), lat.pack(y)
    d = W.wl_blas_dot(lat.ctx, X, Y, W.WL_FULL)
    assert d == complex(np.sum(np.conj(x) * y))
    assert W.wl_blas_norm2(lat.ctx, X, W.WL_FULL) == float(np.sum(np.abs(x) ** 2))
    W.wl_blas_axpy(lat.ctx, -3.0, X, Y, W.WL_FULL)
    assert np.array_equal(lat.unpack(Y).reshape(shp), y - 3 * x)


def test_blas_dot_matches_compensated_sum():
    import math
    dims = (6, 10, 4, 14)
    _, lat = setup(dims)
    x = synth.gaussian_spinor(dims, seed=51)
    y = synth.gaussian_spinor(dims, seed=52)
    d = W.wl_blas_dot(lat.ctx, lat.pack(x), lat.pack(y), W.WL_FULL)
    p = (np.conj(x) * y).ravel()
    want = complex(math.fsum(p.real), math.fsum(p.imag))
    assert abs(d - want) <= 1e-14 * np.sum(np.abs(p))


# ------------------------------------------------------------------ CG
def cg_oracle_ops(u, kappa, phases=AP):
    m = lambda v: orc.dirac(v, u, kappa, phases)
    md = lambda v: orc.dirac(v, u, kappa, phases, dagger=True)
    return m, md


def config1():
    """8^4, kappa 0.12, links exp(0.5 i H) seed 101, Gaussian source seed 102, antiperiodic in t."""
    dims = (8, 8, 8, 8)
    u, lat = setup(dims, eps=0.5, seed=101)
    b = synth.gaussian_spinor(dims, seed=102)
    return dims, u, lat, b, 0.12


@pytest.mark.parametrize("k", [5, 20, 60])
def test_cg_fixed_iterations_match_oracle(k):
    dims, u, lat, b, kappa = config1()
    m, md = cg_oracle_ops(u, kappa)
    x_orc, _ = orc.cg_normal(m, md, b, fixed_iters=k)
    p = W.wl_solver_params_default()
    p.tol = 0.0
    p.maxiter = k
    p.max_restarts = 0
    x = lat.new(W.WL_FULL)
    st, info = W.wl_cg_solve(lat.ctx, x, lat.pack(b), W.WL_OP_D, kappa, params=p)
    assert st == W.WL_NOT_CONVERGED and info[0]["iters"] == k
    err = rel(lat.unpack(x).reshape(b.shape), x_orc)
    print("k", k, "iterate rel diff", err)
    assert err < 1e-13


def test_cg_config1_converges_and_oracle_confirms():
    dims, u, lat, b, kappa = config1()
    m, md = cg_oracle_ops(u, kappa)
    x = lat.new(W.WL_FULL)
    st, info = W.wl_cg_solve(lat.ctx, x, lat.pack(b), W.WL_OP_D, kappa)
    assert st == W.WL_OK
    xs = lat.unpack(x).reshape(b.shape)
    true = rel(md(m(xs)), b)
    x_orc, oinfo = orc.cg_normal(m, md, b, tol=1e-10)
    print("gpu iters", info[0]["iters"], "oracle iters", oinfo["iters"], "oracle-checked residual", true)
    assert true <= 1.05e-10
    assert abs(info[0]["iters"] - oinfo["iters"]) <= 2


def test_cg_even_odd_solves_full_system():
    dims = (6, 10, 4, 14)
    kappa = 0.135
    u, lat = setup(dims, eps=0.2, seed=201)
    eta = synth.gaussian_spinor(dims, seed=202)
    be, bo = orc.eo_split(eta, dims)
    # D x = eta via D_hat: D_hat^+ D_hat x_e = D_hat^+ bhat_e
    bhat = lat.new(W.WL_EVEN)
    W.wl_eo_prepare(lat.ctx, bhat, lat.pack(be, W.WL_EVEN), lat.pack(bo, W.WL_ODD), kappa)
    rhs = lat.new(W.WL_EVEN)
    W.wl_dirac_apply(lat.ctx, rhs, bhat, W.WL_OP_DHAT, True, kappa)
    xe = lat.new(W.WL_EVEN)
    p = W.wl_solver_params_default()
    p.tol = 1e-12
    st, info = W.wl_cg_solve(lat.ctx, xe, rhs, W.WL_OP_DHAT, kappa, params=p)
    assert st == W.WL_OK
    xo = lat.new(W.WL_ODD)
    W.wl_eo_reconstruct(lat.ctx, xo, xe, lat.pack(bo, W.WL_ODD), kappa)
    x = orc.eo_join(lat.unpack(xe, W.WL_EVEN), lat.unpack(xo, W.WL_ODD), dims)
    r = rel(orc.dirac(x, u, kappa, AP), eta)
    print("iters", info[0]["iters"], "||eta - D x|| / ||eta||", r)
    assert r < 1e-9


def test_cg_is_bitwise_reproducible():
    dims, u, lat, b, kappa = config1()
    B = lat.pack(b)
    xs = []
    for _ in range(2):
        x = lat.new(W.WL_FULL)
        W.wl_cg_solve(lat.ctx, x, B, W.WL_OP_D, kappa)
        xs.append(lat.unpack(x))
    assert np.array_equal(xs[0], xs[1])


def test_cg_zero_rhs_and_maxiter_and_breakdown():
    dims = (4, 4, 4, 4)
    u, lat = setup(dims)
    x = lat.new(W.WL_FULL)
    st, info = W.wl_cg_solve(lat.ctx, x, lat.new(W.WL_FULL), W.WL_OP_D, 0.1)
    assert st == W.WL_OK and info[0]["iters"] == 0
    assert not np.any(lat.unpack(x))
    b = synth.gaussian_spinor(dims, seed=61)
    p = W.wl_solver_params_default()
    p.maxiter = 3
    st, info = W.wl_cg_solve(lat.ctx, lat.new(W.WL_FULL), lat.pack(b), W.WL_OP_D, 0.1, params=p)
    assert st == W.WL_NOT_CONVERGED and info[0]["iters"] == 3
    b[1, 1, 1, 1, 2, 1] = np.nan
    st, info = W.wl_cg_solve(lat.ctx, lat.new(W.WL_FULL), lat.pack(b), W.WL_OP_D, 0.1)
    assert st == W.WL_BREAKDOWN


def test_cg_singular_operator_stops_cleanly():
    """U = 1, all directions periodic, kappa = 1/8: D has a zero mode (every constant spinor), so D^+ D x = b
    has no solution for a Gaussian b.  CG must stop by itself (maxiter, or breakdown if <p, A p> vanishes)
    and return; the oracle confirms that the residual of what it returns is at least b's component in the
    null space."""
    dims = (4, 4, 4, 4)
    u = synth.unit_links(dims)
    lat = W.Lattice.create(u, (1, 1, 1, 1))
    try:
        b = synth.gaussian_spinor(dims, seed=67)
        p = W.wl_solver_params_default()
        p.maxiter = 300
        x = lat.new(W.WL_FULL)
        st, info = W.wl_cg_solve(lat.ctx, x, lat.pack(b), W.WL_OP_D, 0.125, params=p)
        assert st in (W.WL_NOT_CONVERGED, W.WL_BREAKDOWN), st
        assert info[0]["iters"] <= p.maxiter
        null = b.mean(axis=(0, 1, 2, 3))  # projection onto the constant spinors
        floor = float(np.linalg.norm(np.broadcast_to(null, b.shape)) / np.linalg.norm(b))
        xs = lat.unpack(x).reshape(b.shape)
        if np.all(np.isfinite(xs)):
            r = orc.dirac(orc.dirac(xs, u, 0.125, (1, 1, 1, 1)), u, 0.125, (1, 1, 1, 1), dagger=True) - b
            assert np.linalg.norm(r) / np.linalg.norm(b) >= 0.99 * floor
        print("status", st, "iters", info[0]["iters"], "null-space floor", floor)
    finally:
        lat.close()


def test_occupancy_cap_keeps_results_bitwise():
    """The occupancy cap only reserves LDS: results are bit for bit those of the uncapped launch."""
    dims = (6, 10, 4, 14)
    ph = random_phases(71)
    u, lat = setup(dims, seed=72, phases=ph)
    stack = np.stack([synth.gaussian_spinor(dims, seed=73 + r).reshape(-1, 4, 3) for r in range(3)])
    for prec in (W.WL_F64, W.WL_F32, W.WL_F16N):
        recon = 12 if prec == W.WL_F16N else 18
        saved = W.wl_ctx_get_launch(lat.ctx, prec)
        try:
            outs = []
            for occ in (0, 1, 3, 8):
                W.wl_ctx_set_launch(lat.ctx, prec, 256, 1, saved[2], saved[3], saved[4], 1, occ)
                o = lat.new(W.WL_FULL, prec, 3)
                W.wl_dirac_apply(lat.ctx, o, lat.pack(stack, W.WL_FULL, prec, 3), W.WL_OP_D, True, 0.13, prec, recon,
                                 3)
                torch.cuda.synchronize()
                outs.append(o.cpu())
            for o in outs[1:]:
                assert torch.equal(o, outs[0])
        finally:
            W.wl_ctx_set_launch(lat.ctx, prec, *saved)


@pytest.mark.parametrize("prec,recon", [(W.WL_F64, 18), (W.WL_F32, 18), (W.WL_F16N, 12)])
@pytest.mark.parametrize("nrhs", [1, 3])
def test_time_sweep_matches_one_point_per_thread(prec, recon, nrhs):
    """The time-sweep kernel (each thread walks `sweep` slices of one column, time neighbours in registers)
    computes every output point with the one-thread-per-point arithmetic: bit for bit equal for sweeps of 1,
    3 and more than Lt slices, on a lattice whose slice does not fill whole blocks, for the hopping term, its
    adjoint and both Dirac operators (epilogues with the x field).  16-bit storage does not use the sweep
    (the setting is ignored), so its results are trivially equal."""
    dims = (6, 10, 4, 14)
    ph = random_phases(87)
    u, lat = setup(dims, seed=88, phases=ph)
    stack = np.stack([synth.gaussian_spinor(dims, seed=89 + r).reshape(-1, 4, 3) for r in range(nrhs)])
    saved = W.wl_ctx_get_launch(lat.ctx, prec)
    outs = {}
    try:
        for sweep in (0, 1, 3, 100):
            W.wl_ctx_set_launch(lat.ctx, prec, 128, 1, 1, 0, -1, 1, 0, sweep)
            inp = lat.pack(stack, W.WL_FULL, prec, nrhs)
            res = []
            for fn in (lambda o: W.wl_dslash_apply(lat.ctx, o, inp, W.WL_FULL, prec, recon, nrhs),
                       lambda o: W.wl_dslash_dagger_apply(lat.ctx, o, inp, W.WL_FULL, prec, recon, nrhs),
                       lambda o: W.wl_dirac_apply(lat.ctx, o, inp, W.WL_OP_D, True, 0.13, prec, recon, nrhs)):
                o = lat.new(W.WL_FULL, prec, nrhs)
                fn(o)
                res.append(o)
            e = lat.new(W.WL_EVEN, prec, nrhs)
            W.wl_dirac_apply(lat.ctx, e, inp[: inp.numel() // 2], W.WL_OP_DHAT, False, 0.13, prec, recon, nrhs)
            res.append(e)
            torch.cuda.synchronize()
            outs[sweep] = [r.cpu() for r in res]
        for sweep in (1, 3, 100):
            for a, b in zip(outs[sweep], outs[0]):
                assert torch.equal(a, b), sweep
    finally:
        W.wl_ctx_set_launch(lat.ctx, prec, *saved)


def test_cg_with_time_sweep():
    """CG whose hopping launches all use the time sweep (norm and residual-update epilogues included):
    every rhs reaches the oracle-restated normal-equation residual."""
    dims, kappa = (6, 10, 4, 14), 0.13
    ph = random_phases(91)
    u, lat = setup(dims, seed=92, phases=ph)
    b = [synth.gaussian_spinor(dims, seed=93 + r) for r in range(2)]
    saved = W.wl_ctx_get_launch(lat.ctx, W.WL_F64)
    try:
        W.wl_ctx_set_launch(lat.ctx, W.WL_F64, 256, 1, 1, W.WL_TCHUNK_AUTO, -1, 1, 0, 4)
        x = lat.new(W.WL_FULL, W.WL_F64, 2)
        st, info = W.wl_cg_solve(lat.ctx, x, lat.pack(np.stack([v.reshape(-1, 4, 3) for v in b]), W.WL_FULL,
                                                      W.WL_F64, 2), W.WL_OP_D, kappa, nrhs=2)
        assert st == W.WL_OK
        xs = lat.unpack(x, W.WL_FULL, W.WL_F64, 2)
        for r in range(2):
            xr = xs[r].reshape(b[r].shape)
            res = orc.dirac(orc.dirac(xr, u, kappa, ph), u, kappa, ph, dagger=True) - b[r]
            assert np.linalg.norm(res) / np.linalg.norm(b[r]) <= 1.05e-10
    finally:
        W.wl_ctx_set_launch(lat.ctx, W.WL_F64, *saved)


def test_cg_free_field_plane_wave_one_iteration():
    dims = (4, 4, 4, 8)
    kappa = 0.12
    u1 = synth.unit_links(dims)
    lat = W.Lattice.create(u1, AP)
    lx, ly, lz, lt = dims
    n = (1, 0, 2, 3)
    theta = (0, 0, 0, np.pi)
    p = [(2 * np.pi * n[m] + theta[m]) / dims[m] for m in range(4)]
    t, z, y, xx = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly), np.arange(lx), indexing="ij")
    rng = np.random.default_rng(2)
    s = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
    b = np.exp(1j * (p[0] * xx + p[1] * y + p[2] * z + p[3] * t))[..., None, None] * s
    lam = (1 - 2 * kappa * np.sum(np.cos(p))) ** 2 + 4 * kappa ** 2 * np.sum(np.sin(p) ** 2)
    x = lat.new(W.WL_FULL)
    prm = W.wl_solver_params_default()
    prm.tol = 1e-12
    st, info = W.wl_cg_solve(lat.ctx, x, lat.pack(b), W.WL_OP_D, kappa, params=prm)
    assert st == W.WL_OK and info[0]["iters"] == 1
    assert rel(lat.unpack(x).reshape(b.shape), b / lam) < 1e-13
    lat.close()


# ------------------------------------------------------------------ launch configurations
@pytest.mark.parametrize("prec", [W.WL_F64, W.WL_F32])
@pytest.mark.parametrize("block,swizzle,tps,tchunk,nt", [(64, 0, 1, 0, 0), (256, 1, 2, 0, 1), (128, 0, 2, 3, -1),
                                                         (192, 1, 1, 4, 1), (64, 1, 2, 5, 0), (256, 1, 1, 1, 1),
                                                         (128, 1, 2, -1, 1), (256, 0, 1, -3, -1), (64, 1, 1, -2, 0),
                                                         (256, 1, 1, W.WL_TCHUNK_YZ, 1), (128, 0, 2, W.WL_TCHUNK_YZ, -1)])
def test_launch_configs_match_oracle(prec, block, swizzle, tps, tchunk, nt):
    dims = (6, 10, 4, 14)
    kappa = 0.13
    ph = random_phases(77)
    u, lat = setup(dims, seed=78, phases=ph)
    saved = W.wl_ctx_get_launch(lat.ctx, prec)
    W.wl_ctx_set_launch(lat.ctx, prec, block, swizzle, tps, tchunk, nt)
    try:
        assert W.wl_ctx_get_launch(lat.ctx, prec) == (block, swizzle, tps, tchunk, nt, 1, 0, 0)
        phi = synth.gaussian_spinor(dims, seed=79)
        for dagger in (False, True):
            want = orc.hop(phi, u, ph, dagger=dagger)
            out = lat.new(W.WL_FULL, prec)
            fn = W.wl_dslash_dagger_apply if dagger else W.wl_dslash_apply
            fn(lat.ctx, out, lat.pack(phi, W.WL_FULL, prec), W.WL_FULL, prec, 18)
            assert rel(lat.unpack(out, W.WL_FULL, prec).reshape(want.shape), want) < TOL[prec]
        # fused epilogue (x + b H in) through the Schur operator
        pe, _ = orc.eo_split(phi, dims)
        want_e = orc.schur(pe, u, kappa, ph, dagger=True)
        oe = lat.new(W.WL_EVEN, prec)
        W.wl_dirac_apply(lat.ctx, oe, lat.pack(pe, W.WL_EVEN, prec), W.WL_OP_DHAT, True, kappa, prec, 18)
        assert rel(lat.unpack(oe, W.WL_EVEN, prec), want_e) < TOL[prec]
        if prec == W.WL_F64:
            # CG uses the fused-norm epilogue: iterates still match the oracle
            b = synth.gaussian_spinor(dims, seed=80)
            m = lambda v: orc.dirac(v, u, kappa, ph)
            md = lambda v: orc.dirac(v, u, kappa, ph, dagger=True)
            x_orc, _ = orc.cg_normal(m, md, b, fixed_iters=15)
            p = W.wl_solver_params_default()
            p.tol, p.maxiter, p.max_restarts = 0.0, 15, 0
            x = lat.new(W.WL_FULL)
            W.wl_cg_solve(lat.ctx, x, lat.pack(b), W.WL_OP_D, kappa, params=p)
            assert rel(lat.unpack(x).reshape(b.shape), x_orc) < 1e-13
    finally:
        W.wl_ctx_set_launch(lat.ctx, prec, *saved)


@pytest.mark.parametrize("prec,recon", [(W.WL_F64, 18), (W.WL_F32, 18), (W.WL_BF16N, 12)])
@pytest.mark.parametrize("dims", [(8, 6, 8, 6), (4, 2, 12, 10), (6, 4, 4, 8)])
def test_processing_orders_give_the_same_bits(prec, recon, dims):
    """The processing order only decides which thread computes which point: the y-z block order,
    the z-ranges and the e/o index order give bit-identical fields (3 right-hand sides, both
    output parities through the Schur operator's fused epilogue too).  (6, 4, 4, 8) has Lz = 4,
    where the y-z blocks are single z-planes."""
    nrhs = 3
    ph = random_phases(83)
    u, lat = setup(dims, seed=84, phases=ph)
    phis = [synth.gaussian_spinor(dims, seed=85 + r) for r in range(nrhs)]
    inp = lat.pack(np.stack([p.reshape(-1, 4, 3) for p in phis]), W.WL_FULL, prec, nrhs)
    ie = lat.pack(np.stack([orc.eo_split(p, dims)[0] for p in phis]), W.WL_EVEN, prec, nrhs)
    saved = W.wl_ctx_get_launch(lat.ctx, prec)
    outs = []
    try:
        for tch in (0, -2, W.WL_TCHUNK_YZ):
            W.wl_ctx_set_launch(lat.ctx, prec, 256, 1, 1, tch)
            out = lat.new(W.WL_FULL, prec, nrhs)
            W.wl_dslash_apply(lat.ctx, out, inp, W.WL_FULL, prec, recon, nrhs=nrhs)
            oe = lat.new(W.WL_EVEN, prec, nrhs)
            W.wl_dirac_apply(lat.ctx, oe, ie, W.WL_OP_DHAT, False, 0.12, prec, recon, nrhs=nrhs)
            torch.cuda.synchronize()
            outs.append((out.cpu(), oe.cpu()))
    finally:
        W.wl_ctx_set_launch(lat.ctx, prec, *saved)
    for o, e in outs[1:]:
        assert torch.equal(o, outs[0][0]) and torch.equal(e, outs[0][1])


@pytest.mark.parametrize("prec,recon", [(W.WL_F64, 18), (W.WL_F32, 12), (W.WL_F16N, 12)])
@pytest.mark.parametrize("nrhs,rpt", [(12, 2), (12, 3), (12, 4), (4, 4), (6, 3)])
def test_rhs_per_thread_matches_one_point_per_thread(prec, recon, nrhs, rpt):
    """rpt > 1 applies each loaded link to rpt right-hand sides.  The arithmetic per output point
    is the same up to the compiler's FMA contraction, so the fields agree to rounding: a few
    units in the last place of the arithmetic (FP64, FP32), or one storage step (FP16 + norm)."""
    dims = (6, 4, 4, 8)
    kappa = 0.12
    ph = random_phases(81)
    u, lat = setup(dims, seed=82, phases=ph)
    stack = np.stack([synth.gaussian_spinor(dims, seed=90 + r).reshape(-1, 4, 3) for r in range(nrhs)])
    saved = W.wl_ctx_get_launch(lat.ctx, prec)
    outs = {}
    try:
        for r_ in (1, rpt):
            W.wl_ctx_set_launch(lat.ctx, prec, 128, 1, 1, 0, -1, r_)
            inp = lat.pack(stack, W.WL_FULL, prec, nrhs)
            o1 = lat.new(W.WL_FULL, prec, nrhs)
            W.wl_dslash_dagger_apply(lat.ctx, o1, inp, W.WL_FULL, prec, recon, nrhs)
            o2 = lat.new(W.WL_FULL, prec, nrhs)
            W.wl_dirac_apply(lat.ctx, o2, inp, W.WL_OP_D, False, kappa, prec, recon, nrhs)
            torch.cuda.synchronize()
            outs[r_] = (o1, o2)
        tol = {W.WL_F64: 1e-15, W.WL_F32: 1e-6, W.WL_F16N: 2e-3}[prec]
        for k in range(2):
            a = lat.unpack(outs[1][k], W.WL_FULL, prec, nrhs)
            b = lat.unpack(outs[rpt][k], W.WL_FULL, prec, nrhs)
            assert rel(b, a) < tol
        if prec == W.WL_F64:
            # the fused-norm epilogue inside CG: iterates of every rhs still match the oracle
            W.wl_ctx_set_launch(lat.ctx, prec, 128, 1, 1, 0, -1, rpt)
            p = W.wl_solver_params_default()
            p.tol, p.maxiter, p.max_restarts = 0.0, 10, 0
            x = lat.new(W.WL_FULL, W.WL_F64, nrhs)
            W.wl_cg_solve(lat.ctx, x, lat.pack(stack, W.WL_FULL, W.WL_F64, nrhs), W.WL_OP_D, kappa, nrhs=nrhs,
                          params=p)
            got = lat.unpack(x, W.WL_FULL, W.WL_F64, nrhs)
            m = lambda v: orc.dirac(v, u, kappa, ph)
            md = lambda v: orc.dirac(v, u, kappa, ph, dagger=True)
            for r in (0, nrhs - 1):
                x_orc, _ = orc.cg_normal(m, md, stack[r].reshape(dims[::-1] + (4, 3)), fixed_iters=10)
                assert rel(got[r].reshape(x_orc.shape), x_orc) < 1e-13
    finally:
        W.wl_ctx_set_launch(lat.ctx, prec, *saved)


def test_launch_config_rejects_bad_values():
    _, lat = setup((4, 4, 4, 4))
    for args in [(W.WL_F64, 32, 0, 1), (W.WL_F64, 320, 0, 1), (W.WL_F64, 256, 0, 3),
                 (W.WL_F64, 256, 0, 1, 0, 2), (W.WL_F64, 256, 0, 1, 0, 0, 5), (W.WL_F64, 256, 0, 2, 0, 0, 2)]:
        with pytest.raises(W.WilsonError) as e:
            W.wl_ctx_set_launch(lat.ctx, *args)
        assert e.value.status == W.WL_ERR_ARG



@pytest.mark.parametrize("prec", [W.WL_F16N, W.WL_BF16N, W.WL_I16N])
def test_two_threads_per_point_16bit(prec):
    """16-bit storage with two threads per point: the two halves agree on the point's norm before
    they encode, so each output equals the one-thread result up to the different summation order
    of the 8 hops (at most one storage step of the site's largest component) and matches the
    oracle to the format's tolerance; the fused-norm epilogue drives a mixed CG to 1e-10."""
    dims = (6, 10, 4, 14)
    kappa = 0.13
    ph = random_phases(83)
    u, lat = setup(dims, seed=84, phases=ph)
    phi = synth.gaussian_spinor(dims, seed=85)
    saved = W.wl_ctx_get_launch(lat.ctx, prec)
    step = {W.WL_F16N: 2.0 ** -10, W.WL_BF16N: 2.0 ** -7, W.WL_I16N: 1.0 / 16383}[prec]
    try:
        res = {}
        for tps in (1, 2):
            W.wl_ctx_set_launch(lat.ctx, prec, 128, 1, tps)
            inp = lat.pack(phi, W.WL_FULL, prec)
            outs = []
            for dagger in (False, True):
                o = lat.new(W.WL_FULL, prec)
                (W.wl_dslash_dagger_apply if dagger else W.wl_dslash_apply)(lat.ctx, o, inp, W.WL_FULL, prec, 12)
                outs.append(o)
            o = lat.new(W.WL_FULL, prec)
            W.wl_dirac_apply(lat.ctx, o, inp, W.WL_OP_D, False, kappa, prec, 12)
            outs.append(o)
            torch.cuda.synchronize()
            res[tps] = [lat.unpack(x, W.WL_FULL, prec).reshape(phi.shape) for x in outs]
        wants = [orc.hop(phi, u, ph), orc.hop(phi, u, ph, dagger=True), orc.dirac(phi, u, kappa, ph)]
        for a, b, want in zip(res[1], res[2], wants):
            smax = np.max(np.abs(np.stack([a.real, a.imag])), axis=(0, -1, -2), keepdims=True)[0]
            assert np.all(np.abs(b - a) <= 2 * step * smax + 1e-30)
            assert rel(b, want) < TOL[prec]
        # mixed CG with the two-thread kernels (norm epilogue, reliable updates) converges
        W.wl_ctx_set_launch(lat.ctx, prec, 128, 1, 2)
        b = synth.gaussian_spinor(dims, seed=86)
        pe, po = orc.eo_split(b, dims)
        p = W.wl_solver_params_default()
        p.prec, p.recon, p.tol = prec, 12, 1e-10
        x = lat.new(W.WL_EVEN)
        st, info = W.wl_cg_solve(lat.ctx, x, lat.pack(pe, W.WL_EVEN), W.WL_OP_DHAT, kappa, params=p)
        assert st == W.WL_OK
        xe = lat.unpack(x, W.WL_EVEN)
        a_ = lambda v: orc.schur(orc.schur(v, u, kappa, ph), u, kappa, ph, dagger=True)
        assert rel(a_(xe), pe) <= 1.05e-10
    finally:
        W.wl_ctx_set_launch(lat.ctx, prec, *saved)
