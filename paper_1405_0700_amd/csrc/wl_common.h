// Internal definitions shared by the kernels of the Wilson library (gfx950).
//
// Complex arithmetic helpers, the storage formats of spinor and link fields,
// the lattice geometry and the block-level FP64 reductions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wilson.h"

namespace wl {

// ------------------------------------------------------------------ complex
template <typename T> struct cpx {
    T re, im;
};

template <typename T> __device__ __forceinline__ cpx<T> mk(T r, T i) { return {r, i}; }
template <typename T> __device__ __forceinline__ cpx<T> operator+(cpx<T> a, cpx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T> __device__ __forceinline__ cpx<T> operator-(cpx<T> a, cpx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T> __device__ __forceinline__ cpx<T> operator-(cpx<T> a) { return {-a.re, -a.im}; }
template <typename T> __device__ __forceinline__ cpx<T> operator*(T s, cpx<T> a) { return {s * a.re, s * a.im}; }
// i * a
template <typename T> __device__ __forceinline__ cpx<T> ti(cpx<T> a) { return {-a.im, a.re}; }
// a * b (the fused multiply-adds are written out, so that every kernel that
// inlines this rounds the same way, whatever the compiler would contract)
template <typename T> __device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b) {
    return {fma(a.re, b.re, -(a.im * b.im)), fma(a.re, b.im, a.im * b.re)};
}
// conj(a) * b
template <typename T> __device__ __forceinline__ cpx<T> cjmul(cpx<T> a, cpx<T> b) {
    return {fma(a.re, b.re, a.im * b.im), fma(a.re, b.im, -(a.im * b.re))};
}
// c + a * b
template <typename T> __device__ __forceinline__ cpx<T> cfma(cpx<T> a, cpx<T> b, cpx<T> c) {
    return {fma(a.re, b.re, fma(-a.im, b.im, c.re)), fma(a.re, b.im, fma(a.im, b.re, c.im))};
}
// c + conj(a) * b
template <typename T> __device__ __forceinline__ cpx<T> cjfma(cpx<T> a, cpx<T> b, cpx<T> c) {
    return {fma(a.re, b.re, fma(a.im, b.im, c.re)), fma(a.re, b.im, fma(-a.im, b.re, c.im))};
}
template <typename T> __device__ __forceinline__ cpx<T> conjg(cpx<T> a) { return {a.re, -a.im}; }

// ------------------------------------------------------------------ 16-bit conversions
// FP16 through the hardware conversion (round to nearest even); BF16 by
// integer rounding of the FP32 bit pattern (round to nearest even, NaN kept).
__device__ __forceinline__ uint16_t f32_to_f16(float f) {
    _Float16 h = (_Float16)f;
    return __builtin_bit_cast(uint16_t, h);
}
__device__ __forceinline__ float f16_to_f32(uint16_t u) { return (float)__builtin_bit_cast(_Float16, u); }
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
    uint32_t u = __builtin_bit_cast(uint32_t, f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);  // quiet NaN
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t u) { return __builtin_bit_cast(float, (uint32_t)u << 16); }

template <int P> struct Half16;
// dec(u) = raw(u) * scale: raw is the stored number, scale the format's fixed factor
template <> struct Half16<WL_F16N> {
    static constexpr float scale = 1.0f;
    __device__ static float raw(uint16_t u) { return f16_to_f32(u); }
    __device__ static float dec(uint16_t u) { return f16_to_f32(u); }
    __device__ static uint16_t enc(float f) { return f32_to_f16(f); }
};
template <> struct Half16<WL_BF16N> {
    static constexpr float scale = 1.0f;
    __device__ static float raw(uint16_t u) { return bf16_to_f32(u); }
    __device__ static float dec(uint16_t u) { return bf16_to_f32(u); }
    __device__ static uint16_t enc(float f) { return f32_to_bf16(f); }
};
// 16-bit fixed point for values in [-1, 1]: q = round(32767 f)
template <> struct Half16<WL_I16N> {
    static constexpr float scale = 1.0f / 32767.0f;
    __device__ static float raw(uint16_t u) { return (float)(int16_t)u; }
    __device__ static float dec(uint16_t u) { return (float)(int16_t)u * (1.0f / 32767.0f); }
    __device__ static uint16_t enc(float f) {
        const float q = fminf(fmaxf(rintf(f * 32767.0f), -32767.0f), 32767.0f);
        return (uint16_t)(int16_t)q;
    }
};

// ------------------------------------------------------------------ spinor storage
// An internal field of one parity holds n = Vh * nrhs "points" (site, rhs),
// rhs fastest.  Points are grouped in blocks of 64 (a wavefront); a block
// stores its points' components as structure-of-arrays of 16-byte units, and
// blocks follow each other, so the loads of one wavefront touch one
// contiguous stretch of memory:
//   F64  : 12 units of double2 (component c)                      192 B / point
//   F32  :  6 units of float4 (components 2k, 2k+1)               96 B / point
//   F16N / BF16N: 3 units of 8 x 16-bit (components 4k .. 4k+3), then the
//          64 float norms of the block                            52 B / point
// Unit k of point i lives at unit index ((i / 64) * NU + k) * 64 + i % 64.
// A field of one parity occupies ceil(n / 64) blocks.
constexpr int BLK = 64;

// Loads of single-use data (the links of an operator application) and stores
// of outputs can carry the non-temporal hint (NT = true), so that they do not
// push the re-read neighbour spinors out of L2.  The hint also keeps them out
// of the Infinity Cache, so it only pays once the working set exceeds it.
typedef double v2d __attribute__((ext_vector_type(2)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v2f __attribute__((ext_vector_type(2)));
typedef unsigned v4u __attribute__((ext_vector_type(4)));
typedef unsigned v2u __attribute__((ext_vector_type(2)));
template <bool NT, typename V> __device__ __forceinline__ V ld_link(const void *p) {
    if constexpr (NT) return __builtin_nontemporal_load((const V *)p);
    else return *(const V *)p;
}
template <bool NT, typename V> __device__ __forceinline__ void st_out(void *p, V v) {
    if constexpr (NT) __builtin_nontemporal_store(v, (V *)p);
    else *(V *)p = v;
}
__device__ __forceinline__ long blk_unit(long i, int nu, int k) { return ((i >> 6) * nu + k) * BLK + (i & 63); }

template <int P> struct SpinorIO;

template <> struct SpinorIO<WL_F64> {
    using real = double;
    static constexpr size_t bytes_per_point = 192;
    __device__ static void load(const void *base, long i, cpx<double> v[12]) {
        const double2 *p = (const double2 *)base + blk_unit(i, 12, 0);
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            double2 d = p[c * BLK];
            v[c] = {d.x, d.y};
        }
    }
    template <bool NT = false> __device__ static void store(void *base, long i, const cpx<double> v[12]) {
        double2 *p = (double2 *)base + blk_unit(i, 12, 0);
#pragma unroll
        for (int c = 0; c < 12; ++c) st_out<NT, v2d>(p + c * BLK, v2d{v[c].re, v[c].im});
    }
    // components 6 hf .. 6 hf + 5 (spins 2 hf, 2 hf + 1)
    __device__ static void load_half(const void *base, long i, int hf, cpx<double> v[6]) {
        const double2 *p = (const double2 *)base + blk_unit(i, 12, 6 * hf);
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            double2 d = p[c * BLK];
            v[c] = {d.x, d.y};
        }
    }
    template <bool NT = false> __device__ static void store_half(void *base, long i, int hf, const cpx<double> v[6]) {
        double2 *p = (double2 *)base + blk_unit(i, 12, 6 * hf);
#pragma unroll
        for (int c = 0; c < 6; ++c) st_out<NT, v2d>(p + c * BLK, v2d{v[c].re, v[c].im});
    }
};

template <> struct SpinorIO<WL_F32> {
    using real = float;
    static constexpr size_t bytes_per_point = 96;
    __device__ static void load(const void *base, long i, cpx<float> v[12]) {
        const float4 *p = (const float4 *)base + blk_unit(i, 6, 0);
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            float4 d = p[k * BLK];
            v[2 * k] = {d.x, d.y};
            v[2 * k + 1] = {d.z, d.w};
        }
    }
    template <bool NT = false> __device__ static void store(void *base, long i, const cpx<float> v[12]) {
        float4 *p = (float4 *)base + blk_unit(i, 6, 0);
#pragma unroll
        for (int k = 0; k < 6; ++k)
            st_out<NT, v4f>(p + k * BLK, v4f{v[2 * k].re, v[2 * k].im, v[2 * k + 1].re, v[2 * k + 1].im});
    }
    __device__ static void load_half(const void *base, long i, int hf, cpx<float> v[6]) {
        const float4 *p = (const float4 *)base + blk_unit(i, 6, 3 * hf);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            float4 d = p[k * BLK];
            v[2 * k] = {d.x, d.y};
            v[2 * k + 1] = {d.z, d.w};
        }
    }
    template <bool NT = false> __device__ static void store_half(void *base, long i, int hf, const cpx<float> v[6]) {
        float4 *p = (float4 *)base + blk_unit(i, 6, 3 * hf);
#pragma unroll
        for (int k = 0; k < 3; ++k)
            st_out<NT, v4f>(p + k * BLK, v4f{v[2 * k].re, v[2 * k].im, v[2 * k + 1].re, v[2 * k + 1].im});
    }
};

// 16-bit storage with a per-point FP32 norm; a block is 3 * 64 uint4 followed
// by 64 floats (3328 bytes).
template <int P> struct SpinorIO16 {
    using real = float;
    static constexpr size_t bytes_per_point = 52;
    static constexpr long block_bytes = 52 * BLK;
    __device__ static const uint4 *units(const void *base, long i) {
        return (const uint4 *)((const char *)base + (i >> 6) * block_bytes) + (i & 63);
    }
    __device__ static float *norm_ptr(const void *base, long i) {
        return (float *)((char *)base + (i >> 6) * block_bytes + 48 * BLK) + (i & 63);
    }
    __device__ static void load(const void *base, long i, cpx<float> v[12]) {
        const uint4 *p = units(base, i);
        const float s = *norm_ptr(base, i);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            uint4 d = p[k * BLK];
            uint32_t w[4] = {d.x, d.y, d.z, d.w};
#pragma unroll
            for (int j = 0; j < 4; ++j)
                v[4 * k + j] = {s * Half16<P>::dec((uint16_t)(w[j] & 0xffffu)),
                                s * Half16<P>::dec((uint16_t)(w[j] >> 16))};
        }
    }
    // The stored numbers (raw, without the norm) and the factor that load()
    // applies to them (the point's norm times the format's fixed scale).
    __device__ static float load_unscaled(const void *base, long i, cpx<float> v[12]) {
        const uint4 *p = units(base, i);
        const float s = *norm_ptr(base, i);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            uint4 d = p[k * BLK];
            uint32_t w[4] = {d.x, d.y, d.z, d.w};
#pragma unroll
            for (int j = 0; j < 4; ++j)
                v[4 * k + j] = {Half16<P>::raw((uint16_t)(w[j] & 0xffffu)), Half16<P>::raw((uint16_t)(w[j] >> 16))};
        }
        return s * Half16<P>::scale;
    }
    template <bool NT = false> __device__ static void store(void *base, long i, const cpx<float> v[12]) {
        uint4 *p = (uint4 *)units(base, i);
        float s = 0.f;
#pragma unroll
        for (int c = 0; c < 12; ++c) s = fmaxf(s, fmaxf(fabsf(v[c].re), fabsf(v[c].im)));
        // a point whose largest component is below the smallest normal float is
        // stored as zero: 1 / s would overflow (such values appear at the edge of
        // the support of a point-source solve, products of ever smaller terms)
        if (!(s >= 1.17549435e-38f)) s = 0.f;
        const float inv = s > 0.f ? 1.0f / s : 0.f;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            uint32_t w[4];
#pragma unroll
            for (int j = 0; j < 4; ++j)
                w[j] = (uint32_t)Half16<P>::enc(v[4 * k + j].re * inv) |
                       ((uint32_t)Half16<P>::enc(v[4 * k + j].im * inv) << 16);
            st_out<NT, v4u>(p + k * BLK, v4u{w[0], w[1], w[2], w[3]});
        }
        st_out<NT, float>(norm_ptr(base, i), s);
    }
    // Spin half hf (components 6 hf .. 6 hf + 5): half 0 is unit 0 and the low 8
    // bytes of unit 1, half 1 the high 8 bytes of unit 1 and unit 2.
    __device__ static void load_half(const void *base, long i, int hf, cpx<float> v[6]) {
        const uint4 *p = units(base, i);
        const float s = *norm_ptr(base, i);
        const uint4 f = p[(hf ? 2 : 0) * BLK];
        const uint2 q = ((const uint2 *)(p + BLK))[hf];
        const uint32_t w[6] = {hf ? q.x : f.x, hf ? q.y : f.y, hf ? f.x : f.z,
                               hf ? f.y : f.w, hf ? f.z : q.x, hf ? f.w : q.y};
#pragma unroll
        for (int j = 0; j < 6; ++j)
            v[j] = {s * Half16<P>::dec((uint16_t)(w[j] & 0xffffu)), s * Half16<P>::dec((uint16_t)(w[j] >> 16))};
    }
    // Stores spin half hf with the point's norm s (the largest component over
    // both halves, found by the caller), encoded exactly as store() does; v is
    // replaced by the values as stored.  The hf = 0 half writes the norm.
    template <bool NT = false>
    __device__ static void store_half_shared(void *base, long i, int hf, cpx<float> v[6], float s) {
        if (!(s >= 1.17549435e-38f)) s = 0.f;
        const float inv = s > 0.f ? 1.0f / s : 0.f;
        uint32_t w[6];
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            const uint16_t lo = Half16<P>::enc(v[j].re * inv), hi = Half16<P>::enc(v[j].im * inv);
            w[j] = (uint32_t)lo | ((uint32_t)hi << 16);
            v[j] = {s * Half16<P>::dec(lo), s * Half16<P>::dec(hi)};
        }
        uint4 *p = (uint4 *)units(base, i);
        const v4u full = hf ? v4u{w[2], w[3], w[4], w[5]} : v4u{w[0], w[1], w[2], w[3]};
        const v2u part = hf ? v2u{w[0], w[1]} : v2u{w[4], w[5]};
        st_out<NT, v4u>(p + (hf ? 2 : 0) * BLK, full);
        st_out<NT, v2u>((v2u *)(p + BLK) + hf, part);
        if (hf == 0) st_out<NT, float>(norm_ptr(base, i), s);
    }
};
template <> struct SpinorIO<WL_F16N> : SpinorIO16<WL_F16N> {};
template <> struct SpinorIO<WL_BF16N> : SpinorIO16<WL_BF16N> {};
template <> struct SpinorIO<WL_I16N> : SpinorIO16<WL_I16N> {};

// ------------------------------------------------------------------ link storage
// Links of one (parity, mu) slab: Vh links in blocks of 64 sites, each block
// structure-of-arrays of 16-byte (or 8-byte) units, like the spinors:
//   F64 18: 9 double2 (row-major entries)                     144 B
//   F64 12: 6 double2 (rows 0 and 1)                           96 B
//   F32 18: 4 float4 (entries 0..7), then 1 float2 (entry 8)   72 B
//   F32 12: 3 float4 (entries 0..5)                            48 B
//   16-bit 12: 1 x 8 halves (entries 0..3), then 1 x 4 halves (4, 5)   24 B
// For 12-real storage the third row is rebuilt as conj(row0 x row1) (valid for
// SU(3)); boundary phases are applied afterwards, outside the link.
template <int P, int R> struct LinkIO;

template <typename T> __device__ __forceinline__ void recon_row2(cpx<T> u[9]) {
    // row2 = conj(row0 x row1)
    u[6] = conjg(cmul(u[1], u[5]) - cmul(u[2], u[4]));
    u[7] = conjg(cmul(u[2], u[3]) - cmul(u[0], u[5]));
    u[8] = conjg(cmul(u[0], u[4]) - cmul(u[1], u[3]));
}

template <int NU> struct LinkIOF64 {
    using real = double;
    static constexpr size_t bytes_per_link = 16 * NU;
    template <bool NT = false> __device__ static void load(const void *base, long i, cpx<double> u[9]) {
        const double2 *p = (const double2 *)base + blk_unit(i, NU, 0);
#pragma unroll
        for (int k = 0; k < NU; ++k) {
            v2d d = ld_link<NT, v2d>(p + k * BLK);
            u[k] = {d.x, d.y};
        }
        if constexpr (NU == 6) recon_row2(u);
    }
    __device__ static void store(void *base, long i, const cpx<double> u[9]) {
        double2 *p = (double2 *)base + blk_unit(i, NU, 0);
#pragma unroll
        for (int k = 0; k < NU; ++k) p[k * BLK] = make_double2(u[k].re, u[k].im);
    }
};
template <> struct LinkIO<WL_F64, 18> : LinkIOF64<9> {};
template <> struct LinkIO<WL_F64, 12> : LinkIOF64<6> {};

template <> struct LinkIO<WL_F32, 18> {
    using real = float;
    static constexpr size_t bytes_per_link = 72;
    // block: 4 * 64 float4, then 64 float2
    template <bool NT = false> __device__ static void load(const void *base, long i, cpx<float> u[9]) {
        const char *b = (const char *)base + (i >> 6) * (72 * BLK);
        const float4 *p = (const float4 *)b + (i & 63);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            v4f d = ld_link<NT, v4f>(p + k * BLK);
            u[2 * k] = {d.x, d.y};
            u[2 * k + 1] = {d.z, d.w};
        }
        v2f e = ld_link<NT, v2f>((const float2 *)(b + 64 * BLK) + (i & 63));
        u[8] = {e.x, e.y};
    }
    __device__ static void store(void *base, long i, const cpx<float> u[9]) {
        char *b = (char *)base + (i >> 6) * (72 * BLK);
        float4 *p = (float4 *)b + (i & 63);
#pragma unroll
        for (int k = 0; k < 4; ++k)
            p[k * BLK] = make_float4(u[2 * k].re, u[2 * k].im, u[2 * k + 1].re, u[2 * k + 1].im);
        ((float2 *)(b + 64 * BLK))[i & 63] = make_float2(u[8].re, u[8].im);
    }
};
template <> struct LinkIO<WL_F32, 12> {
    using real = float;
    static constexpr size_t bytes_per_link = 48;
    template <bool NT = false> __device__ static void load(const void *base, long i, cpx<float> u[9]) {
        const float4 *p = (const float4 *)base + blk_unit(i, 3, 0);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            v4f d = ld_link<NT, v4f>(p + k * BLK);
            u[2 * k] = {d.x, d.y};
            u[2 * k + 1] = {d.z, d.w};
        }
        recon_row2(u);
    }
    __device__ static void store(void *base, long i, const cpx<float> u[9]) {
        float4 *p = (float4 *)base + blk_unit(i, 3, 0);
#pragma unroll
        for (int k = 0; k < 3; ++k)
            p[k * BLK] = make_float4(u[2 * k].re, u[2 * k].im, u[2 * k + 1].re, u[2 * k + 1].im);
    }
};
template <int P> struct LinkIO16 {
    using real = float;
    static constexpr size_t bytes_per_link = 24;
    // block: 64 uint4, then 64 uint2
    template <bool NT = false> __device__ static void load(const void *base, long i, cpx<float> u[9]) {
        const char *b = (const char *)base + (i >> 6) * (24 * BLK);
        v4u a = ld_link<NT, v4u>((const uint4 *)b + (i & 63));
        v2u c = ld_link<NT, v2u>((const uint2 *)(b + 16 * BLK) + (i & 63));
        uint32_t w[6] = {a.x, a.y, a.z, a.w, c.x, c.y};
#pragma unroll
        for (int k = 0; k < 6; ++k)
            u[k] = {Half16<P>::dec((uint16_t)(w[k] & 0xffffu)), Half16<P>::dec((uint16_t)(w[k] >> 16))};
        recon_row2(u);
    }
    __device__ static void store(void *base, long i, const cpx<float> u[9]) {
        uint32_t w[6];
#pragma unroll
        for (int k = 0; k < 6; ++k)
            w[k] = (uint32_t)Half16<P>::enc(u[k].re) | ((uint32_t)Half16<P>::enc(u[k].im) << 16);
        char *b = (char *)base + (i >> 6) * (24 * BLK);
        ((uint4 *)b)[i & 63] = make_uint4(w[0], w[1], w[2], w[3]);
        ((uint2 *)(b + 16 * BLK))[i & 63] = make_uint2(w[4], w[5]);
    }
};
template <> struct LinkIO<WL_F16N, 12> : LinkIO16<WL_F16N> {};
template <> struct LinkIO<WL_BF16N, 12> : LinkIO16<WL_BF16N> {};
template <> struct LinkIO<WL_I16N, 12> : LinkIO16<WL_I16N> {};

// host-side sizes: a field of n points (or a slab of n links) occupies
// ceil(n / 64) blocks
__host__ __device__ inline long padded(long n) { return (n + 63) / 64 * 64; }
inline size_t spinor_point_bytes(int prec) {
    switch (prec) {
    case WL_F64: return 192;
    case WL_F32: return 96;
    default: return 52;
    }
}
inline size_t link_bytes(int prec, int recon) {
    if (prec == WL_F64) return recon == 12 ? 96 : 144;
    if (prec == WL_F32) return recon == 12 ? 48 : 72;
    return 24;
}

// ------------------------------------------------------------------ geometry
// Division of a non-negative 32-bit integer by a divisor d >= 1 fixed at set-up,
// by a multiply-high, an add and shifts instead of the division sequence: the
// round-up method of Granlund and Montgomery ("Division by invariant integers
// using multiplication", 1994): l = ceil(log2 d), m = floor(2^32 (2^l - d) / d) + 1,
// t = mulhi(m, n), q = (t + ((n - t) >> min(l, 1))) >> max(l - 1, 0); exact for
// every 32-bit n (d = 1 gives m = 1, t = 0, q = n).
struct FastDiv {
    uint32_t m;
    int s1, s2;
    int d;
};
inline FastDiv make_fastdiv(int d) {
    int l = 0;
    while ((1LL << l) < d) ++l;
    FastDiv f;
    f.m = (uint32_t)((((unsigned long long)1 << 32) * (unsigned long long)((1LL << l) - d)) / (unsigned long long)d + 1);
    f.s1 = l < 1 ? l : 1;
    f.s2 = l > 1 ? l - 1 : 0;
    f.d = d;
    return f;
}
__host__ __device__ __forceinline__ int fdiv(int n, const FastDiv &f) {
    const uint32_t un = (uint32_t)n;
    const uint32_t t = (uint32_t)(((unsigned long long)f.m * un) >> 32);
    return (int)((t + ((un - t) >> f.s1)) >> f.s2);
}

struct Geom {
    int L[4];      // Lx, Ly, Lz, Lt
    int lxh;       // Lx / 2
    int vh;        // sites per parity
    int sy, sz, st;  // even/odd index strides of y, z, t
    int phase_mask;  // bit mu set if z_mu != 1
    double zr[4], zi[4];
    FastDiv f_lxh, f_ly, f_lz, f_sz;  // division by Lx / 2, Ly, Lz and (Lx / 2) Ly
};

// coordinates of even/odd site i of parity p
__device__ __forceinline__ void eo_coords(const Geom &g, int i, int p, int c[4]) {
    const int r = fdiv(i, g.f_lxh);
    const int xh = i - r * g.lxh;
    const int r2 = fdiv(r, g.f_ly);
    c[1] = r - r2 * g.L[1];
    c[3] = fdiv(r2, g.f_lz);
    c[2] = r2 - c[3] * g.L[2];
    c[0] = 2 * xh + ((c[1] + c[2] + c[3] + p) & 1);
}

// ------------------------------------------------------------------ reductions
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Deterministic sum over the block of `v` (blockDim.x multiple of 64, <= 1024);
// the result is valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double *lds) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if (lane == 0) lds[wid] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < nw; ++w) s += lds[w];
    __syncthreads();
    return s;
}

// Per-right-hand-side block sum: the thread with global point index gid adds
// v to rhs gid % nrhs; out[r * stride] receives the block's sum for rhs r.
// Deterministic (fixed order).  lds must hold blockDim.x doubles; needs
// nrhs <= blockDim.x.  Every thread of the block must call it.
__device__ __forceinline__ void block_sum_rhs(double v, long gid, int nrhs, double *lds, double *out,
                                              long stride) {
    if (nrhs == 1) {
        const double s = block_sum(v, lds);
        if (threadIdx.x == 0) out[0] = s;
        return;
    }
    lds[threadIdx.x] = v;
    __syncthreads();
    if ((int)threadIdx.x < nrhs) {
        const long g0 = gid - threadIdx.x;
        const int r = threadIdx.x;
        const int t0 = (int)(((long)r - g0 % nrhs + nrhs) % nrhs);
        double s = 0.0;
        for (int t = t0; t < (int)blockDim.x; t += nrhs) s += lds[t];
        out[(long)r * stride] = s;
    }
    __syncthreads();
}

// Per-right-hand-side block sum where each thread names its own rhs.
// lds / lrhs must hold blockDim.x entries.  Every thread must call it.
__device__ __forceinline__ void block_sum_by_rhs(double v, int rhs, int nrhs, double *lds, int *lrhs, double *out,
                                                 long stride) {
    if (nrhs == 1) {
        const double s = block_sum(v, lds);
        if (threadIdx.x == 0) out[0] = s;
        return;
    }
    lds[threadIdx.x] = v;
    lrhs[threadIdx.x] = rhs;
    __syncthreads();
    // stage 1: thread t sums right-hand side t % nrhs over slice t / nrhs of the
    // block (q slices of len entries); stage 2: one thread per right-hand side adds
    // its q slice sums.  A fixed order, ~len + q serial steps instead of blockDim.
    const int nt = blockDim.x, q = nt / nrhs, len = (nt + q - 1) / q;
    const int t = threadIdx.x;
    double part = 0.0;
    if (t < q * nrhs) {
        const int r = t % nrhs, k0 = (t / nrhs) * len, k1 = min(k0 + len, nt);
        for (int k = k0; k < k1; ++k)
            if (lrhs[k] == r) part += lds[k];
    }
    __syncthreads();
    if (t < q * nrhs) lds[t] = part;
    __syncthreads();
    if (t < nrhs) {
        double s = 0.0;
        for (int j = 0; j < q; ++j) s += lds[j * nrhs + t];
        out[(long)t * stride] = s;
    }
    __syncthreads();
}

}  // namespace wl
