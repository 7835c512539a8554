// device_common.h -- device helpers shared by the step kernels (kernels.hip)
// and the surrogate's state kernels (surrogate.hip).  Internal.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gsbs {

// -------------------------------------------------------- wave primitives ---
// Prefix operations over the 64 lanes of a wave built from DPP row shifts and
// row broadcasts: plain VALU instructions, no LDS round trip (the HIP shuffle
// intrinsics go through ds_bpermute).  Every lane of the wave must be active.
// DPP controls (GFX9): row_shr:n = 0x110 + n, row_bcast:15 = 0x142,
// row_bcast:31 = 0x143, wave_shr:1 = 0x138.  A lane with no source (or in a row
// the row mask leaves out) receives `ident`.
template <int kCtrl, int kRowMask>
__device__ __forceinline__ int dpp_src(int ident, int v) {
    return __builtin_amdgcn_update_dpp(ident, v, kCtrl, kRowMask, 0xf, false);
}

// Inclusive scan with an associative operation op(int, int) and its identity.
template <class Op>
__device__ __forceinline__ int wave_scan_op(int v, int ident, Op op) {
    v = op(v, dpp_src<0x111, 0xf>(ident, v));
    v = op(v, dpp_src<0x112, 0xf>(ident, v));
    v = op(v, dpp_src<0x114, 0xf>(ident, v));
    v = op(v, dpp_src<0x118, 0xf>(ident, v));
    v = op(v, dpp_src<0x142, 0xa>(ident, v));
    v = op(v, dpp_src<0x143, 0xc>(ident, v));
    return v;
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    return (uint32_t)wave_scan_op((int)v, 0, [](int a, int b) { return (int)((uint32_t)a + (uint32_t)b); });
}
// The value of lane 63 (wave-uniform).
__device__ __forceinline__ int wave_last(int v) { return __builtin_amdgcn_readlane(v, 63); }
__device__ __forceinline__ int wave_min_i(int v) {
    return wave_last(wave_scan_op(v, INT32_MAX, [](int a, int b) { return a < b ? a : b; }));
}
__device__ __forceinline__ int wave_max_i(int v) {
    return wave_last(wave_scan_op(v, INT32_MIN, [](int a, int b) { return a > b ? a : b; }));
}
__device__ __forceinline__ float wave_min_f(float v) {
    return __int_as_float(wave_last(wave_scan_op(__float_as_int(v), __float_as_int(INFINITY), [](int a, int b) {
        return __float_as_int(fminf(__int_as_float(a), __int_as_float(b)));
    })));
}
__device__ __forceinline__ float wave_max_f(float v) {
    return __int_as_float(wave_last(wave_scan_op(__float_as_int(v), __float_as_int(-INFINITY), [](int a, int b) {
        return __float_as_int(fmaxf(__int_as_float(a), __int_as_float(b)));
    })));
}
// The value of the previous lane (lane 0 receives `first`).
__device__ __forceinline__ uint32_t wave_prev(uint32_t v, uint32_t first) {
    return (uint32_t)dpp_src<0x138, 0xf>((int)first, (int)v);
}

// --------------------------------------------------------------- Philox ---
// Full 128-bit product of a 64-bit constant and x from four 32 x 32 + 64
// multiply-adds (v_mad_u64_u32), shared by the low and the high half:
// a b = lo(p00) + 2^32 p10 + 2^64 (hi(p10) + hi(p01) + a1 b1).
template <uint64_t A>
__device__ __forceinline__ void mul128(uint64_t x, uint64_t& lo, uint64_t& hi) {
    constexpr uint32_t a0 = (uint32_t)A, a1 = (uint32_t)(A >> 32);
    const uint32_t x0 = (uint32_t)x, x1 = (uint32_t)(x >> 32);
    const uint64_t p00 = (uint64_t)a0 * x0;
    const uint64_t p01 = (uint64_t)a0 * x1 + (p00 >> 32);
    const uint64_t p10 = (uint64_t)a1 * x0 + (uint32_t)p01;
    lo = (p10 << 32) | (uint32_t)p00;
    hi = (uint64_t)a1 * x1 + (p01 >> 32) + (p10 >> 32);
}

// Philox4x64-10 (Salmon et al., SC'11): multipliers 0xD2E7470EE14C6C93 and
// 0xCA5A826395121157, Weyl increments 0x9E3779B97F4A7C15 and 0xBB67AE8584CAA73B.
__device__ __forceinline__ void philox(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                       uint64_t k0, uint64_t k1, uint64_t out[4]) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B97F4A7C15ull;
            k1 += 0xBB67AE8584CAA73Bull;
        }
        uint64_t lo0, hi0, lo1, hi1;
        mul128<0xD2E7470EE14C6C93ull>(c0, lo0, hi0);
        mul128<0xCA5A826395121157ull>(c2, lo1, hi1);
        const uint64_t n0 = hi1 ^ c1 ^ k0;
        const uint64_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

// PBC 1 (Eq. 1); a jump may exceed one edge, so whole edges are removed first.
__device__ __forceinline__ float wrap_f(float x, float L, float hL, float invL) {
    const float k = floorf(__fmul_rn(__fadd_rn(x, hL), invL));
    x = __fsub_rn(x, __fmul_rn(k, L));
    // selects of plain IEEE operations (no contraction is enabled) keep this branch-free
    x = x >= hL ? x - L : x;
    x = x < -hL ? x + L : x;
    return x;
}

// PBC 2 (Eq. 2).
__device__ __forceinline__ float minimg_f(float d, float L, float hL) {
    const float lo = d - L, hi = d + L;
    return d >= hL ? lo : (d < -hL ? hi : d);
}


// Uniform (k + 1/2) 2^-24 of the top 24 bits of a Philox word, as FP32 (exact
// only up to one rounding: used where no decision hangs on the last bit).
__device__ __forceinline__ float u24_f(uint64_t w) { return ((float)(uint32_t)(w >> 40) + 0.5f) * 0x1p-24f; }

}  // namespace gsbs
