// vkt_mfma_common.h -- pieces shared by the matrix-core ApplyFilter kernels
// (vkt_filter_mfma.hip, vkt_filter_mfma_rp.hip): operand splitting into
// 16-bit pieces, address modes, buffer loads and the output store.
//
// Split precision (16-bit operands, exact FP32 products, FP32 sums):
//   uint8   voxels: exact in fp16 (1 piece) x weights in 2 fp16 pieces;
//   uint16  voxels: hi byte * 256 and lo byte, both exact in fp16 (2 pieces)
//                   x 2 fp16 weight pieces (4 products);
//   float32 voxels: 2 (or 3) bf16 pieces x 2 (or 3) bf16 weight pieces, the
//                   products whose piece orders sum to <= 1 (3 products) or
//                   <= 2 (6 products).
// fp16 weight pieces are taken of w * 2^s, 2^s chosen on the host so that the
// largest |w| lands in [2^14, 2^15); the result is scaled back by 2^-s.
#pragma once

#include "vkt_internal.h"

#include <type_traits>

namespace vkt {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kNT = 256;                     // threads per workgroup (4 waves)
constexpr uint32_t kRsrcWord3 = 0x00020000u; // gfx9-family raw buffer
constexpr uint32_t kOutside = 0x80000000u;   // byte offset that is dropped / reads 0

// Operand pieces and the products kept.
enum PieceMode { kU8 = 0, kU16 = 1, kF32x3 = 2, kF32x6 = 3 };
template <int PM> struct Pieces;
template <> struct Pieces<kU8> {
    static constexpr bool F16 = true;
    static constexpr int PS = 1, NBI = 2, NPROD = 2;
    static constexpr int prod[NPROD][2] = {{0, 0}, {0, 1}};
};
template <> struct Pieces<kU16> {
    static constexpr bool F16 = true;
    static constexpr int PS = 2, NBI = 2, NPROD = 4;
    static constexpr int prod[NPROD][2] = {{0, 0}, {0, 1}, {1, 0}, {1, 1}};
};
template <> struct Pieces<kF32x3> {
    static constexpr bool F16 = false;
    static constexpr int PS = 2, NBI = 2, NPROD = 3;
    static constexpr int prod[NPROD][2] = {{0, 0}, {0, 1}, {1, 0}};
};
template <> struct Pieces<kF32x6> {
    static constexpr bool F16 = false;
    static constexpr int PS = 3, NBI = 3, NPROD = 6;
    static constexpr int prod[NPROD][2] = {{0, 0}, {0, 1}, {1, 0}, {0, 2}, {1, 1}, {2, 0}};
};

__device__ inline int addr_map(int64_t i, int64_t n, int mode)
{
    if (i >= 0 && i < n) return (int)i;
    if (mode == vktAddressModeClamp) return i < 0 ? 0 : (int)(n - 1);
    if (mode == vktAddressModeWrap) {
        int64_t m = i % n;
        return (int)(m < 0 ? m + n : m);
    }
    if (mode == vktAddressModeMirror) {
        const int64_t p = 2 * n;
        int64_t m = i % p;
        if (m < 0) m += p;
        return (int)(m < n ? m : p - 1 - m);
    }
    return -1;
}

__device__ inline uint32_t xcd_remap(uint32_t b, uint32_t n)
{
    const uint32_t q = n / 8, rem = n % 8, xcd = b % 8, idx = b / 8;
    return xcd < rem ? xcd * (q + 1) + idx : rem * (q + 1) + (xcd - rem) * q + idx;
}

template <typename T>
__device__ inline T buf_load(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    if constexpr (sizeof(T) == 1) {
        return (T)__builtin_amdgcn_raw_buffer_load_b8(r, (int)off, 0, 0);
    } else if constexpr (sizeof(T) == 2) {
        return (T)__builtin_amdgcn_raw_buffer_load_b16(r, (int)off, 0, 0);
    } else {
        return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
    }
}

__device__ inline uint16_t f16_bits(float x) { return __builtin_bit_cast(uint16_t, (_Float16)x); }
__device__ inline float f16_val(uint16_t h) { return (float)__builtin_bit_cast(_Float16, h); }
__device__ inline uint16_t bf16_bits(float x) { return __builtin_bit_cast(uint16_t, (__bf16)x); }
__device__ inline float bf16_val(uint16_t h) { return (float)__builtin_bit_cast(__bf16, h); }

// Split one voxel into its 16-bit pieces (bit patterns).
template <int PM, typename T>
__device__ inline void split_voxel(T s, uint16_t* p)
{
    if constexpr (PM == kU8) {
        p[0] = f16_bits((float)s);
    } else if constexpr (PM == kU16) {
        const uint32_t v = s;
        p[0] = f16_bits((float)((v >> 8) << 8));  // multiple of 256 below 2^16: exact
        p[1] = f16_bits((float)(v & 255u));
    } else {
        const float x = (float)s;
        p[0] = bf16_bits(x);
        const float r1 = x - bf16_val(p[0]);
        p[1] = bf16_bits(r1);
        if constexpr (PM == kF32x6) p[2] = bf16_bits(r1 - bf16_val(p[1]));
    }
}

// Split one weight into NBI pieces.
template <int PM>
__device__ inline void split_weight(float w, float scale, uint16_t* p)
{
    if constexpr (Pieces<PM>::F16) {
        const float x = w * scale;  // exact (power of two)
        p[0] = f16_bits(x);
        p[1] = f16_bits(x - f16_val(p[0]));
    } else {
        p[0] = bf16_bits(w);
        const float r1 = w - bf16_val(p[0]);
        p[1] = bf16_bits(r1);
        if constexpr (PM == kF32x6) p[2] = bf16_bits(r1 - bf16_val(p[1]));
    }
}

// Round (integer cells) and store one lane's row of N finished outputs at
// byte offset off: one vector store when the row lies inside the volume and
// is 4-byte aligned, else cell stores for the first nx cells.  Dropped rows
// carry an out-of-range offset.
template <typename T, int N>
__device__ inline void store_row(__amdgpu_buffer_rsrc_t r, uint32_t off, const float (&v)[N],
                                 bool vec, int nx, float unscale)
{
    static_assert(N == 8 || N == 4 || N == 2, "rows of 8, 4 or 2 cells");
    if constexpr (std::is_same<T, float>::value) {
        uint32_t u[N];
#pragma unroll
        for (int i = 0; i < N; ++i) u[i] = __float_as_uint(v[i] * unscale);
        if (vec) {
            if constexpr (N == 2) {
                typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
                __builtin_amdgcn_raw_buffer_store_b64(u32x2{u[0], u[1]}, r, (int)off, 0, 0);
            } else {
#pragma unroll
                for (int h = 0; h < N / 4; ++h)
                    __builtin_amdgcn_raw_buffer_store_b128(
                        u32x4{u[4 * h], u[4 * h + 1], u[4 * h + 2], u[4 * h + 3]}, r,
                        (int)off + 16 * h, 0, 0);
            }
        } else {
#pragma unroll
            for (int i = 0; i < N; ++i)
                __builtin_amdgcn_raw_buffer_store_b32(u[i], r, i < nx ? (int)(off + 4 * i) : (int)kOutside,
                                                      0, 0);
        }
    } else {
        constexpr float kMax = std::is_same<T, uint8_t>::value ? 255.f : 65535.f;
        uint32_t u[N];
#pragma unroll
        for (int i = 0; i < N; ++i)
            // floor(q + 1/2) saturated: truncation of a value clamped to [0, max]
            u[i] = (uint32_t)__builtin_amdgcn_fmed3f(fmaf(v[i], unscale, 0.5f), 0.f, kMax);
        if (vec) {
            typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
            if constexpr (sizeof(T) == 2 && N == 8) {
                __builtin_amdgcn_raw_buffer_store_b128(
                    u32x4{u[0] | (u[1] << 16), u[2] | (u[3] << 16), u[4] | (u[5] << 16),
                          u[6] | (u[7] << 16)},
                    r, (int)off, 0, 0);
            } else if constexpr (sizeof(T) == 2 && N == 4) {
                __builtin_amdgcn_raw_buffer_store_b64(
                    u32x2{u[0] | (u[1] << 16), u[2] | (u[3] << 16)}, r, (int)off, 0, 0);
            } else if constexpr (sizeof(T) == 2) {
                __builtin_amdgcn_raw_buffer_store_b32(u[0] | (u[1] << 16), r, (int)off, 0, 0);
            } else if constexpr (N == 8) {
                __builtin_amdgcn_raw_buffer_store_b64(
                    u32x2{u[0] | (u[1] << 8) | (u[2] << 16) | (u[3] << 24),
                          u[4] | (u[5] << 8) | (u[6] << 16) | (u[7] << 24)},
                    r, (int)off, 0, 0);
            } else if constexpr (N == 4) {
                __builtin_amdgcn_raw_buffer_store_b32(u[0] | (u[1] << 8) | (u[2] << 16) | (u[3] << 24),
                                                      r, (int)off, 0, 0);
            } else {
                __builtin_amdgcn_raw_buffer_store_b16((uint16_t)(u[0] | (u[1] << 8)), r, (int)off,
                                                      0, 0);
            }
        } else {
#pragma unroll
            for (int i = 0; i < N; ++i) {
                const int o = i < nx ? (int)(off + sizeof(T) * i) : (int)kOutside;
                if constexpr (sizeof(T) == 2)
                    __builtin_amdgcn_raw_buffer_store_b16((uint16_t)u[i], r, o, 0, 0);
                else
                    __builtin_amdgcn_raw_buffer_store_b8((uint8_t)u[i], r, o, 0, 0);
            }
        }
    }
}


}  // namespace
}  // namespace vkt
