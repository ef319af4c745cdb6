// vkt_filter_mfma.hip -- ApplyFilter for filters of size k >= 5 on the
// matrix cores: an implicit GEMM with split 16-bit operands and FP32
// accumulation.
//
// Operation (paper Sec. 3.2 "Volume Manipulation"; benchmarked as a Gaussian
// blur, Sec. 4.3):
//   T(x,y,z) = sum_{a,b,c} w[a + k(b + k c)] * s(A(x+a-r), A(y+b-r), A(z+c-r)).
//
// GEMM embedding, per input plane zi (D += A * B on 16x16x32 or 32x32x16
// MFMA tiles):
//   M (rows i)    : consecutive output rows y_i of one x-strip,
//   K (reduction) : (filter row b, input column ax) pairs; the A operand is
//                   the input window s(x_s - r + ax, y_i + b - r, zi), read
//                   straight from the LDS-staged plane (no im2col copy),
//   N (columns j) : (filter plane c, output x-offset xo), j = c * NX + xo;
//                   B[(b, ax)][(c, xo)] = w[c][b][ax - xo] (an x-Toeplitz band
//                   of each filter row, zero outside 0 <= ax - xo < k).
// Column group c of D therefore accumulates the contribution of input plane
// zi to output plane zi - c + r: the k output planes an input plane feeds
// live side by side in D (a z ring).  After each input plane the group
// c = k-1 holds a finished output plane; it is stored and the columns shift
// by NX lanes (group c -> c+1, group 0 restarts at zero).
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
#include "vkt_internal.h"

#include <type_traits>

namespace vkt {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kNT = 256;                     // threads per workgroup (4 waves)
constexpr uint32_t kRsrcWord3 = 0x00020000u; // gfx9-family raw buffer
constexpr uint32_t kOutside = 0x80000000u;   // byte offset that reads 0

// MFMA tile shapes.  RPC = filter rows per K chunk, AXW = input columns per
// filter row in the K dimension, NACC = accumulator registers per lane.
template <int SHAPE> struct Mf;
template <> struct Mf<16> {
    static constexpr int MT = 16, NT = 16, RPC = 4, AXW = 8, NACC = 4;
    using acc_t = f32x4;
};
template <> struct Mf<32> {
    static constexpr int MT = 32, NT = 32, RPC = 1, AXW = 16, NACC = 16;
    using acc_t = f32x16;
};

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

template <typename T, int K, int PM>
struct Cfg {
    using Tin = T;
    using PC = Pieces<PM>;
    static constexpr int SHAPE = K <= 7 ? 16 : 32;
    using M = Mf<SHAPE>;
    static constexpr int R = (K - 1) / 2;
    static constexpr int NX = 2;                                    // output x per strip
    static_assert(K * NX <= M::NT, "column groups exceed the tile");
    static_assert(NX + K - 1 <= M::AXW, "x window exceeds the K slots");
    static constexpr int NCH = SHAPE == 16 ? (K + 3) / 4 : K;      // K chunks
    static constexpr int SX = 16;                                   // strips per workgroup
    static constexpr int SY = SHAPE == 16 ? 4 : 2;                  // row blocks per workgroup
    static constexpr int TX = SX * NX, TY = SY * M::MT;             // 32 x 64 output tile
    static constexpr int PITCH = SHAPE == 16 ? 40 : 48;             // >= NX*(SX-1) + AXW
    static_assert(PITCH >= NX * (SX - 1) + M::AXW, "pitch too small");
    static constexpr int HY = TY + K - 1;                           // staged rows
    static constexpr int NE = (PITCH * HY + kNT - 1) / kNT;         // staged cells / thread
    static constexpr int WS = SX / 4;                               // strips per wave
    static constexpr int MTW = WS * SY;                             // M tiles per wave
};

struct MfmaArgs {
    int32_t X, Y, Z;
    int32_t mode;
    int32_t tz, tiles_x, tiles_y;
    uint32_t nblocks;
    float wscale;     // 2^s applied to weights before fp16 splitting (1 for bf16)
    float unscale;    // 2^-s
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

__device__ inline uint16_t f16_bits(float x)
{
    return __builtin_bit_cast(uint16_t, (_Float16)x);
}
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

template <int SHAPE, bool F16>
__device__ inline typename Mf<SHAPE>::acc_t mfma(u16x8 a, u16x8 b, typename Mf<SHAPE>::acc_t c)
{
    if constexpr (SHAPE == 16) {
        if constexpr (F16)
            return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a),
                                                          __builtin_bit_cast(f16x8, b), c, 0, 0, 0);
        else
            return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                           __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
    } else {
        if constexpr (F16)
            return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a),
                                                          __builtin_bit_cast(f16x8, b), c, 0, 0, 0);
        else
            return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a),
                                                           __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
    }
}

// Shift the accumulator columns right by NX lanes inside each NT-wide column
// group of lanes; the first NX columns become zero.
template <int SHAPE, int NX>
__device__ inline float shift_cols(float v, int lane)
{
    if constexpr (SHAPE == 16) {
        // DPP row_shr:NX inside each row of 16 lanes; bound_ctrl writes 0
        return __builtin_bit_cast(
            float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x110 + NX, 0xf,
                                               0xf, true));
    } else {
        const int src = lane - NX;
        const int r = __builtin_amdgcn_ds_bpermute(src < 0 ? 0 : src * 4, __builtin_bit_cast(int, v));
        return (lane % 32) < NX ? 0.f : __builtin_bit_cast(float, r);
    }
}

template <typename T>
__device__ inline T store_value(float t)
{
    if constexpr (std::is_same<T, float>::value) {
        return t;
    } else {
        constexpr float kMax = std::is_same<T, uint8_t>::value ? 255.f : 65535.f;
        return (T)fminf(fmaxf(floorf(t + 0.5f), 0.f), kMax);
    }
}

template <class C>
__global__ __launch_bounds__(kNT, 1) void filter_mfma_kernel(
    const typename C::Tin* __restrict__ src, typename C::Tin* __restrict__ dst,
    const float* __restrict__ w, MfmaArgs a)
{
    using T = typename C::Tin;
    using PC = typename C::PC;
    using M = typename C::M;
    using acc_t = typename M::acc_t;
    constexpr int K = (C::R * 2) + 1;
    constexpr int R = C::R;
    constexpr int PM = std::is_same<T, uint8_t>::value ? kU8
                       : std::is_same<T, uint16_t>::value ? kU16
                       : (PC::NPROD == 6 ? kF32x6 : kF32x3);
    __shared__ __align__(16) uint16_t lds[2][PC::PS][C::HY * C::PITCH];

    const int t = threadIdx.x, lane = t % 64, wave = t / 64;
    const uint32_t lid = xcd_remap(blockIdx.x, a.nblocks);
    const uint32_t ntiles = (uint32_t)a.tiles_x * (uint32_t)a.tiles_y;
    const int tile = (int)(lid % ntiles), slab = (int)(lid / ntiles);
    const int x0 = (tile % a.tiles_x) * C::TX, y0 = (tile / a.tiles_x) * C::TY;
    const int zb = slab * a.tz, ze = min(zb + a.tz, a.Z);
    const int64_t plane = (int64_t)a.X * a.Y;

    // ---- B operand: x-Toeplitz band of each filter row, split into pieces
    u16x8 B[C::NCH][PC::NBI];
    {
        const int j = lane % M::NT, g = lane / M::NT;
        const int c = j / C::NX, xo = j % C::NX;
#pragma unroll
        for (int q = 0; q < C::NCH; ++q) {
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int b = C::SHAPE == 16 ? q * 4 + g : q;
                const int ax = C::SHAPE == 16 ? e : 8 * g + e;
                const int aa = ax - xo;
                float wv = 0.f;
                if (c < K && b < K && aa >= 0 && aa < K) wv = w[(c * K + b) * K + aa];
                uint16_t p[3];
                split_weight<PM>(wv, a.wscale, p);
#pragma unroll
                for (int bi = 0; bi < PC::NBI; ++bi) B[q][bi][e] = p[bi];
            }
        }
    }

    // ---- staging of the input plane: PITCH x HY cells from (x0 - r, y0 - r)
    uint32_t goff[C::NE];
    int32_t loff[C::NE];
#pragma unroll
    for (int i = 0; i < C::NE; ++i) {
        int e = t + i * kNT;
        if (e >= C::PITCH * C::HY) e = C::PITCH * C::HY - 1;
        const int hy = e / C::PITCH, hx = e - hy * C::PITCH;
        const int gx = addr_map((int64_t)x0 - R + hx, a.X, a.mode);
        const int gy = addr_map((int64_t)y0 - R + hy, a.Y, a.mode);
        // cells past the volume edge that only feed zero weights still read a
        // finite value: clamp mode fetches them, border mode reads zero
        goff[i] = (gx < 0 || gy < 0)
                      ? kOutside
                      : ((uint32_t)gy * (uint32_t)a.X + (uint32_t)gx) * (uint32_t)sizeof(T);
        loff[i] = e;
    }
    const int32_t plane_bytes = (int32_t)(plane * (int64_t)sizeof(T));
    uint16_t stage[C::NE][PC::PS];
    auto gather = [&](int zi) {
        const int gz = addr_map(zi, a.Z, a.mode);
        const char* base = reinterpret_cast<const char*>(src) +
                           (gz < 0 ? 0 : (int64_t)gz * plane_bytes);
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<char*>(base), (short)0, gz < 0 ? 0 : plane_bytes, (int)kRsrcWord3);
#pragma unroll
        for (int i = 0; i < C::NE; ++i) split_voxel<PM>(buf_load<T>(rs, goff[i]), stage[i]);
    };
    auto put = [&](int buf) {
#pragma unroll
        for (int i = 0; i < C::NE; ++i)
#pragma unroll
            for (int ps = 0; ps < PC::PS; ++ps) lds[buf][ps][loff[i]] = stage[i][ps];
    };

    acc_t acc[C::MTW];
#pragma unroll
    for (int m = 0; m < C::MTW; ++m)
#pragma unroll
        for (int r = 0; r < M::NACC; ++r) acc[m][r] = 0.f;

    // lane's A-operand coordinates inside an M tile
    const int ai = lane % M::MT, ag = lane / M::MT;

    const int zi_beg = zb - R, zi_end = ze + R;
    gather(zi_beg);
    put(0);
    __syncthreads();

    for (int zi = zi_beg; zi < zi_end; ++zi) {
        const int cur = (zi - zi_beg) & 1;
        gather(min(zi + 1, zi_end - 1));

#pragma unroll
        for (int m = 0; m < C::MTW; ++m) {
            const int strip = wave * C::WS + m % C::WS, yb = m / C::WS;
            const int col = C::NX * strip + (C::SHAPE == 16 ? 0 : 8 * ag);
#pragma unroll
            for (int q = 0; q < C::NCH; ++q) {
                int b = C::SHAPE == 16 ? q * 4 + ag : q;
                if (b > K - 1) b = K - 1;  // zero weights there; keep A finite
                const int row = yb * M::MT + ai + b;
                u16x8 A[PC::PS];
#pragma unroll
                for (int ps = 0; ps < PC::PS; ++ps) {
                    const uint16_t* p = &lds[cur][ps][row * C::PITCH + col];
                    __builtin_memcpy(&A[ps], p, 16);  // 4-byte aligned 16-byte read
                }
#pragma unroll
                for (int pr = 0; pr < PC::NPROD; ++pr)
                    acc[m] = mfma<C::SHAPE, PC::F16>(A[PC::prod[pr][0]], B[q][PC::prod[pr][1]],
                                                     acc[m]);
            }
        }

        put(cur ^ 1);

        // ---- column group k-1 holds output plane zi - r
        const int zo = zi - R;
        if (zo >= zb) {
            const int j = lane % M::NT;
            const int xo = j - (K - 1) * C::NX;
            if (xo >= 0 && xo < C::NX) {
                T* orow = dst + (int64_t)zo * plane;
#pragma unroll
                for (int m = 0; m < C::MTW; ++m) {
                    const int strip = wave * C::WS + m % C::WS, yb = m / C::WS;
                    const int x = x0 + C::NX * strip + xo;
                    if (x < a.X) {
#pragma unroll
                        for (int r = 0; r < M::NACC; ++r) {
                            const int i = C::SHAPE == 16 ? 4 * (lane / 16) + r
                                                         : 8 * (r / 4) + 4 * (lane / 32) + (r % 4);
                            const int y = y0 + yb * M::MT + i;
                            if (y < a.Y)
                                orow[(int64_t)y * a.X + x] = store_value<T>(acc[m][r] * a.unscale);
                        }
                    }
                }
            }
        }
        // ---- advance the ring
#pragma unroll
        for (int m = 0; m < C::MTW; ++m)
#pragma unroll
            for (int r = 0; r < M::NACC; ++r) acc[m][r] = shift_cols<C::SHAPE, C::NX>(acc[m][r], lane);
        __syncthreads();
    }
}

template <class C>
hipError_t launch_cfg(const FilterJob& j, float wscale, hipStream_t s)
{
    MfmaArgs a{};
    a.X = j.X;
    a.Y = j.Y;
    a.Z = j.Z;
    a.mode = j.mode;
    a.tiles_x = (j.X + C::TX - 1) / C::TX;
    a.tiles_y = (j.Y + C::TY - 1) / C::TY;
    const int64_t ntiles = (int64_t)a.tiles_x * a.tiles_y;
    const int64_t want_slabs = (2048 + ntiles - 1) / ntiles;
    int tz = (int)((j.Z + want_slabs - 1) / want_slabs);
    const int K = j.k;
    const int tz_min = 4 * K;
    if (tz < tz_min) tz = tz_min;
    if (tz > 64) tz = 64;
    if (tz > j.Z) tz = j.Z;
    a.tz = tz;
    const int64_t nb = ntiles * ((j.Z + tz - 1) / tz);
    if (nb > 0x7fffffff) return hipErrorInvalidValue;
    a.nblocks = (uint32_t)nb;
    a.wscale = wscale;
    a.unscale = 1.0f / wscale;
    using T = typename C::Tin;
    hipLaunchKernelGGL((filter_mfma_kernel<C>), dim3((unsigned)nb), dim3(kNT), 0, s,
                       static_cast<const T*>(j.src), static_cast<T*>(j.dst), j.wf, a);
    return hipGetLastError();
}

template <typename T, int PM>
hipError_t dispatch_k(const FilterJob& j, float wscale, hipStream_t s)
{
    switch (j.k) {
    case 5: return launch_cfg<Cfg<T, 5, PM>>(j, wscale, s);
    case 7: return launch_cfg<Cfg<T, 7, PM>>(j, wscale, s);
    case 9: return launch_cfg<Cfg<T, 9, PM>>(j, wscale, s);
    case 11: return launch_cfg<Cfg<T, 11, PM>>(j, wscale, s);
    case 13: return launch_cfg<Cfg<T, 13, PM>>(j, wscale, s);
    case 15: return launch_cfg<Cfg<T, 15, PM>>(j, wscale, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_filter_mfma(const FilterJob& j, bool six_products, hipStream_t s)
{
    switch (j.fmt) {
    case vktDataFormatUInt8: return dispatch_k<uint8_t, kU8>(j, j.wscale, s);
    case vktDataFormatUInt16: return dispatch_k<uint16_t, kU16>(j, j.wscale, s);
    case vktDataFormatFloat32:
        return six_products ? dispatch_k<float, kF32x6>(j, 1.0f, s)
                            : dispatch_k<float, kF32x3>(j, 1.0f, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace vkt
