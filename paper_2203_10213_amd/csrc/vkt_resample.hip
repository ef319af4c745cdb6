// vkt_resample.hip -- Resample (trilinear, cell-centred) and Flip of
// structured volumes.
//
// Paper Sec. 3.2: Resample is a core algorithm that changes the size of a
// volume; Flip is a transform algorithm that mirrors it.  Sec. 4 benchmarks
// both on the structured volumes: a downscale by two on every axis, and a
// flip along the axis of the longest extent.
//
// Resample: destination cell i on an axis of n source and m destination
// cells samples the source at u = (i + 1/2) n / m - 1/2 (cell centres),
// trilinear between the two neighbouring cells, neighbours clamped to the
// volume; integer formats round half-up and saturate.  The position is
// split exactly in integer arithmetic into its cell and its fraction, which
// is rounded once to FP32; the interpolation runs in FP32.  An exact factor of two
// on every axis takes a dedicated path: the mean of each 2 x 2 x 2 block
// (integer formats: (sum + 4) >> 3, exact).
// Flip: dst(x) = src(n - 1 - x) along one axis; in place (dst == src) the
// first half along the axis swaps with the mirrored half.
//
// Both are HBM-bound streams.  Launch shape: threadIdx.x runs along a row
// (cells, or 16-byte chunks on the vector paths), threadIdx.y over rows, the
// grid over row groups with a row-stride loop; blocks are 256 threads whose
// x extent is the power of two covering a row (at most 256), so short rows
// still fill whole wavefronts.  The vector paths (16-byte loads and stores)
// run when rows are whole 16-byte chunks and both buffers are 16-byte
// aligned; otherwise one thread per cell.
#include "vkt_internal.h"

#include <type_traits>

namespace vkt {
namespace {

constexpr int kNT = 256;

struct RowGrid {
    dim3 grid, block;
};

// Blocks of 256 threads: x covers `per_row` items (power of two, <= 256),
// y covers rows; the grid covers the rows once (capped; kernels loop).
RowGrid row_grid(int64_t per_row, int64_t nrows)
{
    int bx = 1;
    while (bx < per_row && bx < kNT) bx *= 2;
    const int by = kNT / bx;
    const int64_t gx = (per_row + bx - 1) / bx;
    int64_t gy = (nrows + by - 1) / by;
    if (gy > 65535) gy = 65535;
    if (gy < 1) gy = 1;
    return {dim3((unsigned)gx, (unsigned)gy), dim3((unsigned)bx, (unsigned)by)};
}

template <typename T>
__device__ inline T from_f(float v)
{
    if constexpr (std::is_same<T, float>::value) {
        return v;
    } else {
        constexpr float kMax = std::is_same<T, uint8_t>::value ? 255.f : 65535.f;
        // floor(v + 1/2) saturated: truncation of v + 1/2 clamped to [0, max]
        return (T)(uint32_t)__builtin_amdgcn_fmed3f(v + 0.5f, 0.f, kMax);
    }
}

// Lower and upper neighbour (clamped) and the weight of the upper one for
// destination cell i of m on an axis of n source cells.  The sample position
// u = (i + 1/2) n / m - 1/2 = ((2i + 1) n - m) / (2m) is split exactly in
// integers: with N = (2i + 1) n + m >= 0 (the numerator plus one
// denominator) and D = 2m, floor(u) = N / D - 1 and the fraction is
// (N mod D) / D, rounded once to FP32.  (32-bit division whenever N fits.)
__device__ inline void lin_axis(int i, int n, int m, int& i0, int& i1, float& f)
{
    const uint64_t N = (uint64_t)(2 * (int64_t)i + 1) * (uint64_t)n + (uint64_t)m;
    const uint64_t D = 2 * (uint64_t)m;
    uint64_t q, rem;
    if (N <= 0xffffffffull && D <= 0xffffffffull) {
        const uint32_t n32 = (uint32_t)N, d32 = (uint32_t)D;
        q = n32 / d32;
        rem = n32 - (uint32_t)q * d32;
    } else {
        q = N / D;
        rem = N - q * D;
    }
    f = (float)rem / (float)D;
    const int64_t a = (int64_t)q - 1;
    i0 = (int)min(max(a, (int64_t)0), (int64_t)n - 1);
    i1 = (int)min(max(a + 1, (int64_t)0), (int64_t)n - 1);
}

__device__ inline float lerp(float a, float b, float t) { return a + t * (b - a); }

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// 16-byte load that is read once (streamed past the caches' reuse sets).
__device__ inline uint4 load_stream(const uint4* p)
{
    const u32x4 v = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(p));
    return make_uint4(v.x, v.y, v.z, v.w);
}

// ---- general trilinear resampling: one destination cell per thread -------
template <typename T>
__global__ __launch_bounds__(kNT) void resample_kernel(const T* __restrict__ src,
                                                       T* __restrict__ dst, int X, int Y, int Z,
                                                       int Xo, int Yo, int Zo, int64_t nrows)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= Xo) return;
    int x0, x1;
    float fx;
    lin_axis(x, X, Xo, x0, x1, fx);
    const int64_t plane = (int64_t)X * Y;
    for (int64_t r = (int64_t)blockIdx.y * blockDim.y + threadIdx.y; r < nrows;
         r += (int64_t)gridDim.y * blockDim.y) {
        const int y = (int)(r % Yo), z = (int)(r / Yo);
        int y0, y1, z0, z1;
        float fy, fz;
        lin_axis(y, Y, Yo, y0, y1, fy);
        lin_axis(z, Z, Zo, z0, z1, fz);
        const T* p0 = src + z0 * plane;
        const T* p1 = src + z1 * plane;
        const int64_t o0 = (int64_t)y0 * X, o1 = (int64_t)y1 * X;
        const float a0 = lerp((float)p0[o0 + x0], (float)p0[o0 + x1], fx);
        const float a1 = lerp((float)p0[o1 + x0], (float)p0[o1 + x1], fx);
        const float b0 = lerp((float)p1[o0 + x0], (float)p1[o0 + x1], fx);
        const float b1 = lerp((float)p1[o1 + x0], (float)p1[o1 + x1], fx);
        dst[r * Xo + x] = from_f<T>(lerp(lerp(a0, a1, fy), lerp(b0, b1, fy), fz));
    }
}

// ---- exact downscale by two: one destination cell per thread -------------
template <typename T>
__global__ __launch_bounds__(kNT) void halve_kernel(const T* __restrict__ src,
                                                    T* __restrict__ dst, int X, int Y, int Xo,
                                                    int Yo, int64_t nrows)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= Xo) return;
    const int64_t plane = (int64_t)X * Y;
    for (int64_t r = (int64_t)blockIdx.y * blockDim.y + threadIdx.y; r < nrows;
         r += (int64_t)gridDim.y * blockDim.y) {
        const int y = (int)(r % Yo), z = (int)(r / Yo);
        const T* s0 = src + (2 * z) * plane + (int64_t)(2 * y) * X + 2 * x;
        const T* rows[4] = {s0, s0 + X, s0 + plane, s0 + plane + X};
        if constexpr (std::is_same<T, float>::value) {
            float s = 0.f;
#pragma unroll
            for (int i = 0; i < 4; ++i) s += rows[i][0] + rows[i][1];
            dst[r * Xo + x] = s * 0.125f;
        } else {
            uint32_t s = 0;
#pragma unroll
            for (int i = 0; i < 4; ++i) s += (uint32_t)rows[i][0] + (uint32_t)rows[i][1];
            dst[r * Xo + x] = (T)((s + 4u) >> 3);  // floor(mean + 1/2), exact
        }
    }
}

// ---- exact downscale by two, 16 destination bytes per thread -------------
// Destination row (y, z) averages source rows 2y, 2y + 1 of planes 2z,
// 2z + 1; a thread reads 32 bytes (a, b) of each of those 4 rows.  Integer
// cells are summed in SIMD-within-a-register lanes (u8: two 16-bit lanes
// per dword, at most 8 * 255 each; u16: one 32-bit sum per cell pair).
template <typename T>
__device__ inline void halve_chunk(const uint4 (&a)[4], const uint4 (&b)[4], uint4& out)
{
    if constexpr (std::is_same<T, float>::value) {
        float o[4];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            float s0 = 0.f, s1 = 0.f;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const uint4 v = h ? b[i] : a[i];
                s0 += __uint_as_float(v.x) + __uint_as_float(v.y);
                s1 += __uint_as_float(v.z) + __uint_as_float(v.w);
            }
            o[2 * h] = s0 * 0.125f;
            o[2 * h + 1] = s1 * 0.125f;
        }
        out = make_uint4(__float_as_uint(o[0]), __float_as_uint(o[1]), __float_as_uint(o[2]),
                         __float_as_uint(o[3]));
    } else if constexpr (std::is_same<T, uint16_t>::value) {
        uint32_t s[8] = {};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint32_t w[8] = {a[i].x, a[i].y, a[i].z, a[i].w, b[i].x, b[i].y, b[i].z, b[i].w};
#pragma unroll
            for (int j = 0; j < 8; ++j) s[j] += (w[j] & 0xFFFFu) + (w[j] >> 16);
        }
        uint32_t o[4];
#pragma unroll
        for (int m = 0; m < 4; ++m)
            o[m] = ((s[2 * m] + 4u) >> 3) | (((s[2 * m + 1] + 4u) >> 3) << 16);
        out = make_uint4(o[0], o[1], o[2], o[3]);
    } else {
        // dword j of the 32 source bytes holds x = 4j..4j+3: its two 16-bit
        // lanes collect destination cells 2j and 2j+1
        uint32_t s[8] = {};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint32_t w[8] = {a[i].x, a[i].y, a[i].z, a[i].w, b[i].x, b[i].y, b[i].z, b[i].w};
#pragma unroll
            for (int j = 0; j < 8; ++j) s[j] += (w[j] & 0x00FF00FFu) + ((w[j] >> 8) & 0x00FF00FFu);
        }
        uint32_t o[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            // (lane + 4) >> 3 in both lanes; the low lane's upper bits take
            // spill from the high lane, masked off
            const uint32_t p = ((s[2 * m] + 0x00040004u) >> 3) & 0x00FF00FFu;
            const uint32_t q = ((s[2 * m + 1] + 0x00040004u) >> 3) & 0x00FF00FFu;
            o[m] = (p & 0xFFu) | ((p >> 8) & 0xFF00u) | ((q & 0xFFu) << 16) | ((q << 8) & 0xFF000000u);
        }
        out = make_uint4(o[0], o[1], o[2], o[3]);
    }
}

template <typename T>
__global__ __launch_bounds__(kNT) void halve_vec_kernel(const uint4* __restrict__ src,
                                                        uint4* __restrict__ dst, int cpr,
                                                        int Yo, int64_t nrows)
{
    // cpr: 16-byte chunks per destination row; a source row has 2 cpr
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cpr) return;
    const int64_t srow = 2 * (int64_t)cpr;        // chunks per source row
    const int64_t splane = srow * 2 * Yo;         // chunks per source plane
    for (int64_t r = (int64_t)blockIdx.y * blockDim.y + threadIdx.y; r < nrows;
         r += (int64_t)gridDim.y * blockDim.y) {
        const int y = (int)(r % Yo), z = (int)(r / Yo);
        const uint4* s0 = src + (2 * z) * splane + (2 * y) * srow + 2 * c;
        const uint4* rows[4] = {s0, s0 + srow, s0 + splane, s0 + splane + srow};
        uint4 a[4], b[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            a[i] = load_stream(rows[i]);
            b[i] = load_stream(rows[i] + 1);
        }
        uint4 o;
        halve_chunk<T>(a, b, o);
        dst[r * cpr + c] = o;
    }
}

// ---- Flip ----------------------------------------------------------------
// One cell per thread.  Out of place: every cell; in place: the cells with
// coordinate < n / 2 along the axis swap with their mirror (the middle cell
// of an odd axis stays).  Xs / Ys: cells per row / rows per plane iterated.
template <typename T>
__global__ __launch_bounds__(kNT) void flip_kernel(const T* src, T* dst, int X, int Y, int Z,
                                                   int Xs, int Ys, int64_t nrows, int axis,
                                                   int inplace)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= Xs) return;
    const int mx = axis == 0 ? X - 1 - x : x;
    for (int64_t r = (int64_t)blockIdx.y * blockDim.y + threadIdx.y; r < nrows;
         r += (int64_t)gridDim.y * blockDim.y) {
        const int y = (int)(r % Ys), z = (int)(r / Ys);
        const int my = axis == 1 ? Y - 1 - y : y;
        const int mz = axis == 2 ? Z - 1 - z : z;
        const int64_t o = ((int64_t)z * Y + y) * X + x;
        const int64_t m = ((int64_t)mz * Y + my) * X + mx;
        if (inplace) {
            const T a = dst[o], b = dst[m];
            dst[o] = b;
            dst[m] = a;
        } else {
            dst[o] = src[m];
        }
    }
}

// The cells of a 16-byte chunk in reverse order.
template <typename T>
__device__ inline uint4 reverse_chunk(uint4 v)
{
    if constexpr (std::is_same<T, float>::value) {
        return make_uint4(v.w, v.z, v.y, v.x);
    } else if constexpr (std::is_same<T, uint16_t>::value) {
        auto sw = [](uint32_t u) { return (u >> 16) | (u << 16); };
        return make_uint4(sw(v.w), sw(v.z), sw(v.y), sw(v.x));
    } else {
        return make_uint4(__builtin_bswap32(v.w), __builtin_bswap32(v.z),
                          __builtin_bswap32(v.y), __builtin_bswap32(v.x));
    }
}

// 16-byte chunks per thread; rows are cpr whole chunks.  Along x, chunk c
// of a row comes from chunk cpr - 1 - c with its cells reversed; along y or
// z whole chunks move between mirrored rows.  In place along x only the
// first ceil(cpr / 2) chunks are visited (the middle chunk of an odd count
// is reversed by itself); along y or z only the first half of the rows.
template <typename T>
__global__ __launch_bounds__(kNT) void flip_vec_kernel(const uint4* src, uint4* dst, int cpr,
                                                       int Y, int Z, int cs, int Ys,
                                                       int64_t nrows, int axis, int inplace)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cs) return;
    const int mc = axis == 0 ? cpr - 1 - c : c;
    for (int64_t r = (int64_t)blockIdx.y * blockDim.y + threadIdx.y; r < nrows;
         r += (int64_t)gridDim.y * blockDim.y) {
        const int y = (int)(r % Ys), z = (int)(r / Ys);
        const int my = axis == 1 ? Y - 1 - y : y;
        const int mz = axis == 2 ? Z - 1 - z : z;
        const int64_t o = ((int64_t)z * Y + y) * cpr + c;
        const int64_t m = ((int64_t)mz * Y + my) * cpr + mc;
        if (inplace) {
            const uint4 a = dst[o], b = dst[m];
            dst[o] = axis == 0 ? reverse_chunk<T>(b) : b;
            dst[m] = axis == 0 ? reverse_chunk<T>(a) : a;
        } else {
            const uint4 b = load_stream(src + m);
            dst[o] = axis == 0 ? reverse_chunk<T>(b) : b;
        }
    }
}

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

template <typename T>
hipError_t resample_t(const void* src, void* dst, const int32_t in[3], const int32_t out[3],
                      hipStream_t s)
{
    const int64_t nrows = (int64_t)out[1] * out[2];
    const bool halve = in[0] == 2 * out[0] && in[1] == 2 * out[1] && in[2] == 2 * out[2];
    if (halve && ((int64_t)out[0] * sizeof(T)) % 16 == 0 && aligned16(src) && aligned16(dst)) {
        const int cpr = (int)((int64_t)out[0] * sizeof(T) / 16);
        const RowGrid g = row_grid(cpr, nrows);
        hipLaunchKernelGGL((halve_vec_kernel<T>), g.grid, g.block, 0, s,
                           static_cast<const uint4*>(src), static_cast<uint4*>(dst), cpr, out[1],
                           nrows);
    } else if (halve) {
        const RowGrid g = row_grid(out[0], nrows);
        hipLaunchKernelGGL((halve_kernel<T>), g.grid, g.block, 0, s, static_cast<const T*>(src),
                           static_cast<T*>(dst), in[0], in[1], out[0], out[1], nrows);
    } else {
        const RowGrid g = row_grid(out[0], nrows);
        hipLaunchKernelGGL((resample_kernel<T>), g.grid, g.block, 0, s,
                           static_cast<const T*>(src), static_cast<T*>(dst), in[0], in[1], in[2],
                           out[0], out[1], out[2], nrows);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t flip_t(const void* src, void* dst, const int32_t d[3], int axis, hipStream_t s)
{
    const bool inplace = src == dst;
    // rows per plane and planes iterated (in place along y / z: first half)
    const int Ys = (inplace && axis == 1) ? d[1] / 2 : d[1];
    const int Zs = (inplace && axis == 2) ? d[2] / 2 : d[2];
    const int64_t nrows = (int64_t)Ys * Zs;
    if (((int64_t)d[0] * sizeof(T)) % 16 == 0 && aligned16(src) && aligned16(dst)) {
        const int cpr = (int)((int64_t)d[0] * sizeof(T) / 16);
        const int cs = (inplace && axis == 0) ? (cpr + 1) / 2 : cpr;
        if (nrows == 0) return hipSuccess;
        const RowGrid g = row_grid(cs, nrows);
        hipLaunchKernelGGL((flip_vec_kernel<T>), g.grid, g.block, 0, s,
                           static_cast<const uint4*>(src), static_cast<uint4*>(dst), cpr, d[1],
                           d[2], cs, Ys, nrows, axis, inplace ? 1 : 0);
    } else {
        const int Xs = (inplace && axis == 0) ? d[0] / 2 : d[0];
        if (nrows == 0 || Xs == 0) return hipSuccess;  // in place along one cell
        const RowGrid g = row_grid(Xs, nrows);
        hipLaunchKernelGGL((flip_kernel<T>), g.grid, g.block, 0, s, static_cast<const T*>(src),
                           static_cast<T*>(dst), d[0], d[1], d[2], Xs, Ys, nrows, axis,
                           inplace ? 1 : 0);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_resample(const void* src, void* dst, vktDataFormat f, const int32_t in[3],
                           const int32_t out[3], hipStream_t s)
{
    switch (f) {
    case vktDataFormatUInt8: return resample_t<uint8_t>(src, dst, in, out, s);
    case vktDataFormatUInt16: return resample_t<uint16_t>(src, dst, in, out, s);
    case vktDataFormatFloat32: return resample_t<float>(src, dst, in, out, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_flip(const void* src, void* dst, vktDataFormat f, const int32_t dims[3],
                       int axis, hipStream_t s)
{
    switch (f) {
    case vktDataFormatUInt8: return flip_t<uint8_t>(src, dst, dims, axis, s);
    case vktDataFormatUInt16: return flip_t<uint16_t>(src, dst, dims, axis, s);
    case vktDataFormatFloat32: return flip_t<float>(src, dst, dims, axis, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace vkt
