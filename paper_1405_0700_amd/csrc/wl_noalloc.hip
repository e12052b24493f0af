// C ABI, allocation-free entry point: the dot product of wl_blas_dot with its
// partial sums in a static device array instead of the context's workspace, and
// its result left in device memory, so that it can run where memory cannot be
// allocated (graph capture, tight loops).
//
// The array `scratch` exists once per device for the life of the process.  In
// host code its name is only a stand-in: the device address of each device's
// copy is looked up with hipGetSymbolAddress when the first context is created
// on that device (scratch_setup, called by wl_ctx_create with the device
// current) and kept in g_scratch; kernels get that address as an argument.
#include <mutex>

#include "wl_internal.h"

namespace {
constexpr long SCRATCH_DOUBLES = 1L << 20;  // 8 MiB per device
__device__ __align__(256) double scratch[SCRATCH_DOUBLES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double *g_scratch[MAX_DEVICES] = {};

// out[0] = sum_r vals[r], out[1] = sum_r vals[nrhs + r], summed in the order and
// precision wl_blas_dot uses on the host
__global__ void k_sum_over_rhs(const double *vals, int nrhs, double *out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double re = 0.0, im = 0.0;
    for (int r = 0; r < nrhs; ++r) {
        re += vals[r];
        im += vals[nrhs + r];
    }
    out[0] = re;
    out[1] = im;
}
}  // namespace

// Called by wl_ctx_create with `device` current: looks up this device's copy of
// the scratch array once.
wl_status wli::scratch_setup(int device) {
    if (device < 0 || device >= MAX_DEVICES) return fail(WL_ERR_UNSUPPORTED, "device %d beyond %d", device, MAX_DEVICES);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch[device]) return WL_OK;
    void *ptr = nullptr;
    hipError_t e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
        (void)hipGetLastError();
        return fail(WL_ERR_HIP, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
    }
    g_scratch[device] = (double *)ptr;
    return WL_OK;
}

extern "C" wl_status wl_blas_dot_noalloc(const wl_ctx *c, const void *x, const void *y, wl_subset subset,
                                         wl_prec prec, int nrhs, double *result_dev, void *stream) {
    g_err.clear();
    wl_status st = check_field_args(c, subset, prec, nrhs);
    if (st) return st;
    if (!x || !y || !result_dev || !aligned16(x) || !aligned16(y) || ((uintptr_t)result_dev & 7u))
        return fail(WL_ERR_ARG, "null or misaligned pointer");
    double *buf = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (c->device >= 0 && c->device < MAX_DEVICES) buf = g_scratch[c->device];
    }
    if (!buf) return fail(WL_ERR_HIP, "no scratch address for device %d", c->device);
    const int nh = subset == WL_FULL ? 2 : 1;
    VecArgs v = vec_args(c, prec, nrhs);
    const long nblk = blas_blocks(v.n) * nh;  // blocks of the dot kernel, each leaving one partial per value
    const long need = 2L * nrhs * nblk + 2L * nrhs;
    if (need > SCRATCH_DOUBLES)
        return fail(WL_ERR_ARG, "%ld partial sums exceed the static scratch of %ld doubles (%d rhs of %ld points)",
                    need, SCRATCH_DOUBLES, nrhs, (long)c->Vh * nh);
    const size_t hb = half_bytes(c, prec, nrhs);
    set_vec(v, 0, x, hb);
    set_vec(v, 1, y, hb);
    v.partials = buf;
    v.part_stride = nblk;
    hipStream_t s = (hipStream_t)stream;
    double *vals = buf + 2L * nrhs * nblk;
    HIP_TRY(blas_dot(prec, v, nh, s));
    HIP_TRY(reduce_rows(buf, nblk, nblk, 2 * nrhs, vals, s));
    hipLaunchKernelGGL(k_sum_over_rhs, dim3(1), dim3(64), 0, s, vals, nrhs, result_dev);
    HIP_TRY(hipGetLastError());
    return WL_OK;
}
