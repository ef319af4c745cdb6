// vkt_filter_sep.hip -- ApplyFilter for rank-1 (separable) filters,
// w[c][b][a] = t[c] v[b] u[a], as three one-dimensional passes: 3k
// multiply-adds per output instead of k^3.
//
// Operation (paper Sec. 3.2 "Volume Manipulation": a faster implementation
// of a filter must keep its behaviour; the benchmarked Gaussian blur of
// Sec. 4.3 is separable):
//   T(x,y,z) = sum_c t[c] sum_b v[b] sum_a u[a] s(A(x+a-r), A(y+b-r), A(z+c-r)),
// stored like ApplyFilter.  Integer filters are factored exactly into
// integer factors; the host admits them only when every partial sum stays an
// exact integer in FP32, so the stored quotient is the dense one.
//
// Mapping to gfx950 (same tiling as the vector kernel: 256 threads, 64 x 32
// output tile, 4 x 2 outputs per thread, z-slab marching):
//  * each input plane's halo tile is staged in LDS as FP32, double buffered,
//    with the loads of the plane after next in flight;
//  * x pass: the 64-wide rows of the (32 + 2r)-row halo are filtered with u
//    into a second LDS buffer, also double buffered (4 outputs per thread
//    and row, 16-byte reads); one barrier per plane separates the passes;
//  * y pass: each thread filters its 4 x 2 outputs' columns with v;
//  * z pass: the plane's result enters an input-stationary ring of k partial
//    sums with weights t (slots outside the slab are skipped); the oldest is
//    a finished output.  The z loop is unrolled by k so the ring entries
//    stay in fixed registers.
// The three factor vectors (16 floats each, zero padded) are brought into
// SGPRs by explicit scalar loads: once per tile-slab for k <= 7, else one
// per pass.
#include "vkt_internal.h"

#include <type_traits>
#include <utility>

namespace vkt {
namespace {

constexpr int kBX = 16, kBY = 16, kNT = kBX * kBY;
constexpr int kVX = 4, kVY = 2;
constexpr int kTX = kBX * kVX, kTY = kBY * kVY;  // 64 x 32 tile

template <int K>
struct GeoS {
    static constexpr int R = (K - 1) / 2;
    static constexpr int HX = kTX + 2 * R;                // staged row width
    static constexpr int HY = kTY + 2 * R;                // staged rows
    static constexpr int P = (HX + 3) & ~3;               // staged row pitch (floats)
    static constexpr int NE = (HX * HY + kNT - 1) / kNT;  // staged cells per thread
    static constexpr int XW = kVX + K - 1;                // x-pass window
    static constexpr int XR = (XW + 3) / 4;               // 16-byte reads per window
    static constexpr int A_CELLS = HY * P;                // one staged plane
    static constexpr int B_CELLS = HY * kTX;              // x-pass result
    static constexpr int NXR = (HY + kBY - 1) / kBY;      // x-pass rows per thread
    static_assert(4 * (kBX - 1) + 4 * XR <= P, "x window exceeds the pitch");
};

constexpr uint32_t kRsrcWord3 = 0x00020000u;  // gfx9-family raw buffer
constexpr uint32_t kOutside = 0x80000000u;    // byte offset that reads 0

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
__device__ inline float buf_load(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    if constexpr (sizeof(T) == 1)
        return (float)__builtin_amdgcn_raw_buffer_load_b8(r, (int)off, 0, 0);
    else if constexpr (sizeof(T) == 2)
        return (float)__builtin_amdgcn_raw_buffer_load_b16(r, (int)off, 0, 0);
    else
        return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
}

// 16 factor weights into SGPRs; one explicit scalar load that waits for its
// data (keeps exactly one factor vector live, see the vector kernel).
__device__ inline void load_factor(const float* p, float (&f)[16])
{
    typedef uint32_t v16 __attribute__((ext_vector_type(16)));
    // the address is uniform; readfirstlane keeps it in SGPRs even where
    // register pressure would otherwise leave a copy in VGPRs
    // (readfirstlane returns int: widen through uint32_t, not by sign)
    const uint64_t a = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)a);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(a >> 32));
    const uint64_t sa = (uint64_t)lo | ((uint64_t)hi << 32);
    v16 r;
    asm volatile("s_load_dwordx16 %0, %1, 0x0\n\ts_waitcnt lgkmcnt(0)" : "=&s"(r) : "s"(sa));
#pragma unroll
    for (int q = 0; q < 16; ++q) f[q] = __uint_as_float(r[q]);
}

template <typename F, int... I>
__device__ __attribute__((always_inline)) inline void static_for_impl(
    F& f, std::integer_sequence<int, I...>)
{
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __attribute__((always_inline)) inline void static_for(F&& f)
{
    static_for_impl(f, std::make_integer_sequence<int, N>{});
}

__device__ inline uint32_t udiv(uint32_t n, UDiv d)
{
    const uint32_t t = __umulhi(d.m, n);
    return (t + ((n - t) >> d.sh1)) >> d.sh2;
}

// Stored value of one finished output (T exact integer for integer filters).
template <typename T>
__device__ __attribute__((always_inline)) inline T finish(float acc, const VolDesc& a)
{
    if constexpr (std::is_same<T, float>::value) {
        return a.epi == kEpiFloatDiv ? acc * a.inv_D : acc;
    } else {
        constexpr int kMax = std::is_same<T, uint8_t>::value ? 255 : 65535;
        if (a.epi == kEpiIntDiv) {
            const int32_t t = (int32_t)acc;
            if (t < 0) return (T)0;
            const uint32_t q = udiv(2u * (uint32_t)t + (uint32_t)a.D, a.div2D);
            return (T)(q > (uint32_t)kMax ? (uint32_t)kMax : q);
        }
        const float q = floorf(acc + 0.5f);
        return (T)fminf(fmaxf(q, 0.f), (float)kMax);
    }
}

// One tile-slab; f holds the factors u | v | t at offsets 0, 16, 32.
template <typename T, int K>
__device__ __attribute__((always_inline)) inline void sep_tile(const VolDesc& a, const float* __restrict__ f, int tile, int slab,
                         float* lds)
{
    using G = GeoS<K>;
    constexpr int R = G::R;
    const T* __restrict__ src = static_cast<const T*>(a.src);
    T* __restrict__ dst = static_cast<T*>(a.dst);

    const int t = threadIdx.x, tx = t % kBX, ty = t / kBX;
    const int x0 = a.rx0 + (tile % a.tiles_x) * kTX, y0 = a.ry0 + (tile / a.tiles_x) * kTY;
    const int zb = a.rz0 + slab * a.tz, ze = min(zb + a.tz, a.rz1);
    const int64_t plane = (int64_t)a.X * a.Y;
    // x-pass results, double buffered by plane parity like the staged
    // planes: with both double buffered, one barrier per plane suffices (the
    // x pass of plane p + 1 writes the other buffer while slower waves still
    // read plane p's; plane p + 2 reuses it only after the barrier of p + 1)
    float* const bx0 = lds + 2 * G::A_CELLS;

    uint32_t goff[G::NE];
    int32_t loff[G::NE];
#pragma unroll
    for (int i = 0; i < G::NE; ++i) {
        int e = t + i * kNT;
        if (e >= G::HX * G::HY) e = G::HX * G::HY - 1;  // duplicate write of the last cell
        const int hy = e / G::HX, hx = e - hy * G::HX;
        const int gx = addr_map((int64_t)x0 - R + hx, a.X, a.mode);
        const int gy = addr_map((int64_t)y0 - R + hy, a.Y, a.mode);
        goff[i] = (gx < 0 || gy < 0)
                      ? kOutside
                      : ((uint32_t)gy * (uint32_t)a.X + (uint32_t)gx) * (uint32_t)sizeof(T);
        loff[i] = hy * G::P + hx;
    }
    const int32_t plane_bytes = (int32_t)(plane * (int64_t)sizeof(T));  // < 2^31 (host check)
    float stage[G::NE];
    auto gather = [&](int zi) __attribute__((always_inline)) {
        const int gz = addr_map(zi, a.Z, a.mode);  // -1 only for border: a zero plane
        const char* base = reinterpret_cast<const char*>(src) +
                           (gz < 0 ? 0 : (int64_t)gz * plane_bytes);
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<char*>(base), (short)0, gz < 0 ? 0 : plane_bytes, (int)kRsrcWord3);
#pragma unroll
        for (int i = 0; i < G::NE; ++i) stage[i] = buf_load<T>(rs, goff[i]);
    };
    auto put = [&](float* buf) __attribute__((always_inline)) {
#pragma unroll
        for (int i = 0; i < G::NE; ++i) buf[loff[i]] = stage[i];
    };

    // z ring in fixed registers: the z loop is unrolled by K, and at plane
    // p = zi - zi_beg the ring entry of age c (output plane zi - c + r) sits
    // in slot (c - p) mod K, so no entry moves between planes
    float acc[K][kVY][kVX];

    // k <= 7: the three factor vectors stay in SGPRs for the whole
    // tile-slab; larger k loads each one before its pass (48 live weights
    // would spill SGPRs)
    constexpr bool kHoist = K <= 7;
    float u[16], v[16], tw[16];
    if constexpr (kHoist) {
        load_factor(f, u);
        load_factor(f + 16, v);
        load_factor(f + 32, tw);
    }

    const int zi_beg = zb - R, zi_end = ze + R;
    gather(zi_beg);
    put(lds);
    if (zi_beg + 1 < zi_end) gather(zi_beg + 1);
    __syncthreads();

    const int ox = x0 + kVX * tx, oy = y0 + kVY * ty;
    const bool vec = a.vec_ok && ox + kVX <= a.rx1;

    auto step = [&](int zi, auto U) __attribute__((always_inline)) {
        constexpr int P = decltype(U)::value;  // plane index mod K
        const int cur = (zi - zi_beg) & 1;
        const float* A = lds + cur * G::A_CELLS;
        float* const bx = bx0 + cur * G::B_CELLS;

        // ---- x pass over all staged rows: bx[row][x] = sum_a u[a] A[row][x + a]
        if constexpr (!kHoist) load_factor(f, u);
#pragma unroll
        for (int i = 0; i < G::NXR; ++i) {
            const int row = ty + kBY * i;
            if (row < G::HY) {
                float wdw[4 * G::XR];
#pragma unroll
                for (int q = 0; q < G::XR; ++q) {
                    const float4 v4 =
                        *reinterpret_cast<const float4*>(A + row * G::P + kVX * tx + 4 * q);
                    wdw[4 * q + 0] = v4.x;
                    wdw[4 * q + 1] = v4.y;
                    wdw[4 * q + 2] = v4.z;
                    wdw[4 * q + 3] = v4.w;
                }
                float h[kVX];
#pragma unroll
                for (int vx = 0; vx < kVX; ++vx) {
                    h[vx] = u[0] * wdw[vx];
#pragma unroll
                    for (int aa = 1; aa < K; ++aa) h[vx] = fmaf(u[aa], wdw[vx + aa], h[vx]);
                }
                *reinterpret_cast<float4*>(bx + row * kTX + kVX * tx) =
                    make_float4(h[0], h[1], h[2], h[3]);
            }
        }
        // next plane into the other staging buffer (read two barriers later)
        if (zi + 1 < zi_end) put(lds + (cur ^ 1) * G::A_CELLS);
        if (zi + 2 < zi_end) gather(zi + 2);
        __syncthreads();

        // ---- y pass: p[vy][vx] = sum_b v[b] bx[2 ty + vy + b][4 tx + vx],
        // streaming the k + 1 rows (row j feeds output row vy through v[j - vy])
        float pv[kVY][kVX];
        if constexpr (!kHoist) load_factor(f + 16, v);
#pragma unroll
        for (int j = 0; j < kVY + K - 1; ++j) {
            const float4 v4 = *reinterpret_cast<const float4*>(bx + (kVY * ty + j) * kTX + kVX * tx);
            const float row[kVX] = {v4.x, v4.y, v4.z, v4.w};
#pragma unroll
            for (int vy = 0; vy < kVY; ++vy) {
                const int b = j - vy;
                if (b < 0 || b >= K) continue;
#pragma unroll
                for (int vx = 0; vx < kVX; ++vx)
                    pv[vy][vx] = b == 0 ? v[0] * row[vx] : fmaf(v[b], row[vx], pv[vy][vx]);
            }
        }
        // ---- z pass: age c feeds output plane zi - c + r; age 0 starts its
        // sum (a slot it reuses was stored or is never stored)
        const int c_lo = max(0, zi + R - ze + 1), c_hi = min(K - 1, zi + R - zb);
        if constexpr (!kHoist) load_factor(f + 32, tw);
#pragma unroll
        for (int c = 0; c < K; ++c) {
            if (c < c_lo || c > c_hi) continue;
            const int slot = ((c - P) % K + K) % K;
#pragma unroll
            for (int vy = 0; vy < kVY; ++vy)
#pragma unroll
                for (int vx = 0; vx < kVX; ++vx)
                    acc[slot][vy][vx] = c == 0 ? tw[0] * pv[vy][vx]
                                               : fmaf(tw[c], pv[vy][vx], acc[slot][vy][vx]);
        }

        // ---- the oldest entry (age K - 1) is output plane zo = zi - r
        const int zo = zi - R;
        if (zo >= zb) {
            constexpr int old = ((K - 1 - P) % K + K) % K;
            T* orow = dst + (int64_t)zo * plane;
#pragma unroll
            for (int vy = 0; vy < kVY; ++vy) {
                const int y = oy + vy;
                if (y >= a.ry1) continue;
                T* o = orow + (int64_t)y * a.X + ox;
                T r4[kVX];
#pragma unroll
                for (int vx = 0; vx < kVX; ++vx) r4[vx] = finish<T>(acc[old][vy][vx], a);
                if (vec) {
                    if constexpr (sizeof(T) == 1) {
                        *reinterpret_cast<uchar4*>(o) = make_uchar4(r4[0], r4[1], r4[2], r4[3]);
                    } else if constexpr (sizeof(T) == 2) {
                        *reinterpret_cast<ushort4*>(o) = make_ushort4(r4[0], r4[1], r4[2], r4[3]);
                    } else {
                        *reinterpret_cast<float4*>(o) = make_float4(r4[0], r4[1], r4[2], r4[3]);
                    }
                } else {
#pragma unroll
                    for (int vx = 0; vx < kVX; ++vx)
                        if (ox + vx < a.rx1) o[vx] = r4[vx];
                }
            }
        }
    };

    for (int zi = zi_beg; zi < zi_end; zi += K) {
        static_for<K>([&](auto U) {
            if (zi + decltype(U)::value < zi_end) step(zi + decltype(U)::value, U);
        });
    }
}

template <typename T, int K>
__global__ __launch_bounds__(kNT) void filter_sep_kernel(VolDesc a, const float* __restrict__ f,
                                                         uint32_t nblocks)
{
    __shared__ __align__(16) float lds[2 * GeoS<K>::A_CELLS + 2 * GeoS<K>::B_CELLS];
    const uint32_t lid = xcd_remap(blockIdx.x, nblocks);
    const uint32_t ntiles = (uint32_t)a.tiles_x * (uint32_t)a.tiles_y;
    sep_tile<T, K>(a, f, (int)(lid % ntiles), (int)(lid / ntiles), lds);
}

template <typename T, int K>
hipError_t launch_k(const FilterJob& j, hipStream_t s)
{
    const ClassGeom g{kTX, kTY, 4 > 2 * K ? 4 : 2 * K};
    const int RX = j.roi[3] - j.roi[0], RY = j.roi[4] - j.roi[1], RZ = j.roi[5] - j.roi[2];
    const int64_t ntiles = (int64_t)((RX + g.tx - 1) / g.tx) * ((RY + g.ty - 1) / g.ty);
    const void* fn = (const void*)&filter_sep_kernel<T, K>;
    const int tz = plan_tz(ntiles, RZ, K, 1, 128, resident_wgs(fn), 1);
    const VolDesc a = make_desc(j, tz, g);
    const int64_t nb = ntiles * ((RZ + tz - 1) / tz);
    if (nb > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL((filter_sep_kernel<T, K>), dim3((unsigned)nb), dim3(kNT), 0, s, a, j.wsep,
                       (uint32_t)nb);
    return hipGetLastError();
}

template <typename T>
hipError_t dispatch_k(const FilterJob& j, hipStream_t s)
{
    switch (j.k) {
    case 1: return launch_k<T, 1>(j, s);
    case 3: return launch_k<T, 3>(j, s);
    case 5: return launch_k<T, 5>(j, s);
    case 7: return launch_k<T, 7>(j, s);
    case 9: return launch_k<T, 9>(j, s);
    case 11: return launch_k<T, 11>(j, s);
    case 13: return launch_k<T, 13>(j, s);
    case 15: return launch_k<T, 15>(j, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_filter_sep(const FilterJob& j, hipStream_t s)
{
    switch (j.fmt) {
    case vktDataFormatUInt8: return dispatch_k<uint8_t>(j, s);
    case vktDataFormatUInt16: return dispatch_k<uint16_t>(j, s);
    case vktDataFormatFloat32: return dispatch_k<float>(j, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace vkt
