// Device helpers shared by the MFMA tile kernels (tile.h) and the small
// kernels of kernels.hip: compile-time loops, the device scalar block, and
// the low-precision operand formats (storage traits and conversions).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>

#include "kernels.h"

namespace psvt {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

template <typename F, int... Is>
__device__ __forceinline__ void static_for_impl(F &&f, std::integer_sequence<int, Is...>) {
    (f(std::integral_constant<int, Is>{}), ...);
}
// f(0), f(1), ..., f(N-1) with compile-time constant arguments
template <int N, typename F>
__device__ __forceinline__ void static_for(F &&f) {
    static_for_impl(f, std::make_integer_sequence<int, N>{});
}

__device__ __forceinline__ float scal(const Scalars *sc, int idx) { return idx >= 0 ? sc->f[idx] : 1.0f; }

// --------------------------------------------------------- operand types

// Storage of one GEMM operand.  Every type moves in 16-byte chunks; an LDS
// row holds 8 chunks (128 bytes) of the k dimension plus a 16-byte pad.
template <int ET>
struct Op;
template <>
struct Op<OP_F32> {
    typedef float T;
    static constexpr int EPC = 4;  // elements per 16-byte chunk
};
template <>
struct Op<OP_BF16> {
    typedef uint16_t T;
    static constexpr int EPC = 8;
};
template <>
struct Op<OP_BF16X3> {
    typedef uint16_t T;
    static constexpr int EPC = 8;
};
template <>
struct Op<OP_FP8> {
    typedef uint8_t T;
    static constexpr int EPC = 16;
};

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int intx8 __attribute__((ext_vector_type(8)));

// float -> bfloat16, round to nearest even (inputs are finite)
__device__ __forceinline__ uint16_t to_bf16(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// float -> OCP FP8 e4m3 (gfx950 hardware conversion, round to nearest even),
// saturated to the largest finite value 448.
__device__ __forceinline__ uint8_t to_fp8(float x) {
    x = fminf(fmaxf(x, -448.0f), 448.0f);
    return (uint8_t)(__builtin_amdgcn_cvt_pk_fp8_f32(x, 0.0f, 0, false) & 0xFF);
}

// Store one value in a low-precision copy; split bf16 writes hi at idx and
// the residual lo at idx + plane.
__device__ __forceinline__ void store_lp(void *base, int type, int64_t idx, float v, int64_t plane = 0) {
    if (type == OP_BF16) {
        ((uint16_t *)base)[idx] = to_bf16(v);
    } else if (type == OP_BF16X3) {
        const uint16_t hi = to_bf16(v);
        const float hv = __uint_as_float((uint32_t)hi << 16);
        ((uint16_t *)base)[idx] = hi;
        ((uint16_t *)base)[idx + plane] = to_bf16(v - hv);
    } else {
        ((uint8_t *)base)[idx] = to_fp8(v);
    }
}

// Four consecutive elements idx .. idx+3 of a low-precision copy in one store
// per plane (8 bytes of bf16, 4 of fp8) when the address allows it; the same
// bytes as four store_lp calls.
__device__ __forceinline__ void store_lp4(void *base, int type, int64_t idx, const float v[4], float scale,
                                          int64_t plane = 0) {
    const int esz = type == OP_FP8 ? 1 : 2;
    const uintptr_t addr = (uintptr_t)base + (uintptr_t)(idx * esz);
    const uintptr_t addr_lo = (uintptr_t)base + (uintptr_t)((idx + plane) * esz);
    if ((addr & (4 * esz - 1)) != 0 || (type == OP_BF16X3 && (addr_lo & 7) != 0)) {
#pragma unroll
        for (int e = 0; e < 4; ++e) store_lp(base, type, idx + e, v[e] * scale, plane);
        return;
    }
    if (type == OP_FP8) {
        float c[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) c[e] = fminf(fmaxf(v[e] * scale, -448.0f), 448.0f);
        int w = __builtin_amdgcn_cvt_pk_fp8_f32(c[0], c[1], 0, false);
        w = __builtin_amdgcn_cvt_pk_fp8_f32(c[2], c[3], w, true);
        *(uint32_t *)addr = (uint32_t)w;
        return;
    }
    uint16_t hi[4], lo[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const float x = v[e] * scale;
        hi[e] = to_bf16(x);
        lo[e] = to_bf16(x - __uint_as_float((uint32_t)hi[e] << 16));
    }
    *(uint2 *)addr = make_uint2(hi[0] | ((uint32_t)hi[1] << 16), hi[2] | ((uint32_t)hi[3] << 16));
    if (type == OP_BF16X3)
        *(uint2 *)addr_lo = make_uint2(lo[0] | ((uint32_t)lo[1] << 16), lo[2] | ((uint32_t)lo[3] << 16));
}

}  // namespace psvt
