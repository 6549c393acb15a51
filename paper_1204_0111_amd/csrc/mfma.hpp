// Matrix-core primitives shared by the front and solve kernels.
//
// A complex tile product is four real products per 16 x 16 x 4 step (there
// is no complex MFMA instruction), or three in the solve passes, which add
// the operands' parts first: FP32 MFMA for complex64 and FP64 MFMA for
// complex128, accumulating in the same precision.  Operand layout of the
// 16 x 16 x 4 instructions: lane l supplies A(l % 16, k) and B(k, l % 16) for
// k = l / 16; register r of lane l receives D(mfma_out_row(l / 16, r), l % 16).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace hsw {

typedef float mf4 __attribute__((ext_vector_type(4)));
typedef double md4 __attribute__((ext_vector_type(4)));
template <typename T> struct MfmaAcc;
template <> struct MfmaAcc<float> { typedef mf4 type; };
template <> struct MfmaAcc<double> { typedef md4 type; };
__device__ inline mf4 mfma4(float a, float b, mf4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ inline md4 mfma4(double a, double b, md4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Output row held by lane group lk = lane / 16 in register r: FP32 places
// four consecutive rows per lane group, FP64 interleaves them (row lk + 4 r).
template <typename T> __device__ inline int mfma_out_row(int lk, int r);
template <> __device__ inline int mfma_out_row<float>(int lk, int r) { return 4 * lk + r; }
template <> __device__ inline int mfma_out_row<double>(int lk, int r) { return lk + 4 * r; }

// Buffer loads through a resource descriptor of `bytes` bytes at p: a load
// whose offset lies past the end (offsets are unsigned, so a negative one
// does too) returns zeros instead of touching memory.  Dword 3 selects the
// 32-bit data format that untyped loads need on this architecture.
typedef __amdgpu_buffer_rsrc_t BufRsrc;
__device__ inline BufRsrc buf_rsrc(const void* p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}
__device__ inline int buf_load_i32(BufRsrc r, uint32_t off) {
    return (int)__builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0);
}
template <typename T> struct BufCx;
template <> struct BufCx<float> {
    typedef float v2 __attribute__((ext_vector_type(2)));
    __device__ static inline void load(BufRsrc r, uint32_t off, float& re, float& im) {
        const v2 v = __builtin_bit_cast(v2, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
        re = v.x;
        im = v.y;
    }
};
template <> struct BufCx<double> {
    typedef double v2 __attribute__((ext_vector_type(2)));
    __device__ static inline void load(BufRsrc r, uint32_t off, double& re, double& im) {
        const v2 v = __builtin_bit_cast(v2, __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, 0));
        re = v.x;
        im = v.y;
    }
};

}  // namespace hsw
