// vkt_filter_valu.hip -- ApplyFilter on the vector ALUs (FP32 FMA, or exact
// 24-bit integer multiply-add for integer-weight filters on integer cells).
//
// Operation (paper Sec. 3.2 "Volume Manipulation"; benchmarked as a Gaussian
// blur of structured volumes in Sec. 4.3): for every output cell,
//   T(x,y,z) = sum_{a,b,c} w[a + k(b + k c)] * s(A(x+a-r), A(y+b-r), A(z+c-r)).
//
// Mapping to gfx950:
//  * A workgroup of 256 threads owns a 64 x 32 (x, y) output tile and marches
//    through a z-slab of output planes.  Each input plane of the slab, with an
//    r-wide halo in x and y, is gathered once from HBM (the address mode is
//    applied to halo coordinates only, through per-thread offsets computed
//    once per workgroup) and staged in LDS, double buffered.
//  * Input-stationary z ring: a thread owns 4 (x) x 2 (y) output columns and
//    keeps k partial sums per output, one per output plane zi - c + r that the
//    current input plane zi contributes to.  Each input plane is read from LDS
//    once per thread (16-byte reads of its (4+k-1)-wide row windows) and
//    feeds all k^3 taps; after the plane, the finished output plane (the
//    ring's oldest) is rounded and stored and the ring advances.
//  * Workgroups are numbered XCD-aware so that tiles adjacent in x/y at the
//    same z run on the same XCD and share its L2 for the halo re-reads.
#include "vkt_internal.h"

#include <type_traits>

namespace vkt {
namespace {

constexpr int kBX = 16, kBY = 16, kNT = kBX * kBY;  // threads per workgroup
constexpr int kVX = 4, kVY = 2;                      // outputs per thread
constexpr int kTX = kBX * kVX, kTY = kBY * kVY;      // 64 x 32 tile

template <int K>
struct Geo {
    static constexpr int R = (K - 1) / 2;
    static constexpr int HX = kTX + 2 * R;             // halo tile width
    static constexpr int HY = kTY + 2 * R;             // halo tile height
    static constexpr int P = (HX + 3) & ~3;            // LDS row pitch (cells)
    static constexpr int NE = (HX * HY + kNT - 1) / kNT;  // halo cells / thread
    static constexpr int WX = kVX + K - 1;             // row window per thread
    static constexpr int NR = (WX + 3) / 4;            // 16-byte reads per row
    static_assert(4 * (kBX - 1) + 4 * NR <= P, "row window exceeds LDS pitch");
};

// Address mode on one axis; -1 means "outside, reads zero" (border).
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

// Workgroup id -> logical tile id such that consecutive logical ids land on
// the same XCD (the dispatcher deals workgroups to the 8 XCDs round-robin).
__device__ inline uint32_t xcd_remap(uint32_t b, uint32_t n)
{
    const uint32_t q = n / 8, rem = n % 8, xcd = b % 8, idx = b / 8;
    return xcd < rem ? xcd * (q + 1) + idx : rem * (q + 1) + (xcd - rem) * q + idx;
}

template <typename T> __device__ inline float to_f(T v) { return (float)v; }

template <bool IACC> struct AccT { using type = float; };
template <> struct AccT<true> { using type = int32_t; };

__device__ inline float mac(float w, float v, float acc) { return fmaf(w, v, acc); }
__device__ inline int32_t mac(int32_t w, int32_t v, int32_t acc)
{
    return __mul24(w, v) + acc;  // |w| < 2^23 and cells < 2^16: exact
}

__device__ inline uint32_t udiv(uint32_t n, UDiv d)
{
    const uint32_t t = __umulhi(d.m, n);
    return (t + ((n - t) >> d.sh1)) >> d.sh2;
}

// Stored value of one finished output.
template <typename T, bool IACC>
__device__ inline T finish(typename AccT<IACC>::type acc, const FilterJob& j)
{
    if constexpr (std::is_same<T, float>::value) {
        return j.int_filter ? acc * j.inv_D : acc;
    } else {
        constexpr float kMax = std::is_same<T, uint8_t>::value ? 255.f : 65535.f;
        if constexpr (IACC) {
            // floor((2T + D) / (2D)), exact; T < 0 always stores 0
            if (acc < 0) return (T)0;
            const uint32_t q = udiv(2u * (uint32_t)acc + (uint32_t)j.D, j.div2D);
            return (T)(q > (uint32_t)kMax ? (uint32_t)kMax : q);
        } else {
            const float q = floorf(acc + 0.5f);
            return (T)fminf(fmaxf(q, 0.f), kMax);
        }
    }
}

template <typename T, int K, bool IACC>
__global__ __launch_bounds__(kNT) void filter_valu_kernel(
    const T* __restrict__ src, T* __restrict__ dst,
    const typename AccT<IACC>::type* __restrict__ w, FilterJob j, int32_t tz,
    int32_t tiles_x, int32_t tiles_y, uint32_t nblocks)
{
    using G = Geo<K>;
    using Acc = typename AccT<IACC>::type;
    constexpr int R = G::R;
    __shared__ __align__(16) Acc lds[2][G::HY * G::P];

    const int t = threadIdx.x, tx = t % kBX, ty = t / kBX;
    const uint32_t lid = xcd_remap(blockIdx.x, nblocks);
    const uint32_t ntiles = (uint32_t)tiles_x * (uint32_t)tiles_y;
    const int tile = (int)(lid % ntiles), slab = (int)(lid / ntiles);
    const int x0 = (tile % tiles_x) * kTX, y0 = (tile / tiles_x) * kTY;
    const int zb = slab * tz, ze = min(zb + tz, j.Z);
    const int64_t plane = (int64_t)j.X * j.Y;

    // Halo gather offsets: same (x, y) cells for every plane of the slab.
    int32_t goff[G::NE];  // in-plane source offset, -1 = zero cell
    int32_t loff[G::NE];  // LDS slot, -1 = none
#pragma unroll
    for (int i = 0; i < G::NE; ++i) {
        const int e = t + i * kNT;
        if (e < G::HX * G::HY) {
            const int hy = e / G::HX, hx = e - hy * G::HX;
            const int gx = addr_map((int64_t)x0 - R + hx, j.X, j.mode);
            const int gy = addr_map((int64_t)y0 - R + hy, j.Y, j.mode);
            goff[i] = (gx < 0 || gy < 0) ? -1 : gy * j.X + gx;
            loff[i] = hy * G::P + hx;
        } else {
            goff[i] = -1;
            loff[i] = -1;
        }
    }

    Acc stage[G::NE];
    auto gather = [&](int zi) {
        const int gz = addr_map(zi, j.Z, j.mode);
        const T* base = src + (gz < 0 ? 0 : (int64_t)gz * plane);
#pragma unroll
        for (int i = 0; i < G::NE; ++i) {
            Acc v = 0;
            if (gz >= 0 && goff[i] >= 0) {
                if constexpr (IACC) v = (int32_t)base[goff[i]];
                else v = to_f(base[goff[i]]);
            }
            stage[i] = v;
        }
    };
    auto put = [&](Acc* buf) {
#pragma unroll
        for (int i = 0; i < G::NE; ++i)
            if (loff[i] >= 0) buf[loff[i]] = stage[i];
    };

    Acc acc[K][kVY][kVX];
#pragma unroll
    for (int c = 0; c < K; ++c)
#pragma unroll
        for (int vy = 0; vy < kVY; ++vy)
#pragma unroll
            for (int vx = 0; vx < kVX; ++vx) acc[c][vy][vx] = 0;

    const int zi_beg = zb - R, zi_end = ze + R;  // input planes [beg, end)
    gather(zi_beg);
    put(lds[0]);
    __syncthreads();

    const int ox = x0 + kVX * tx, oy = y0 + kVY * ty;
    for (int zi = zi_beg; zi < zi_end; ++zi) {
        const int cur = (zi - zi_beg) & 1;
        const bool more = zi + 1 < zi_end;
        if (more) gather(zi + 1);

        // ---- all k^3 taps of input plane zi, for the k output planes it feeds
        const Acc* buf = lds[cur];
        constexpr int NROW = kVY + K - 1;
constexpr int kRowUnroll = K <= 5 ? NROW : 1;
#pragma unroll kRowUnroll
        for (int jr = 0; jr < NROW; ++jr) {
            Acc v[G::NR * 4];
            const Acc* row = buf + (kVY * ty + jr) * G::P + kVX * tx;
#pragma unroll
            for (int q = 0; q < G::NR; ++q) {
                const auto u = *reinterpret_cast<const typename std::conditional<
                    IACC, int4, float4>::type*>(row + 4 * q);
                v[4 * q + 0] = u.x; v[4 * q + 1] = u.y;
                v[4 * q + 2] = u.z; v[4 * q + 3] = u.w;
            }
#pragma unroll
            for (int vy = 0; vy < kVY; ++vy) {
                const int b = jr - vy;
                if (b < 0 || b >= K) continue;
#pragma unroll
                for (int c = 0; c < K; ++c)
#pragma unroll
                    for (int a = 0; a < K; ++a) {
                        const Acc wv = w[(c * K + b) * K + a];
#pragma unroll
                        for (int vx = 0; vx < kVX; ++vx)
                            acc[c][vy][vx] = mac(wv, v[vx + a], acc[c][vy][vx]);
                    }
            }
        }

        if (more) put(lds[cur ^ 1]);

        // ---- the ring's oldest plane zo = zi - r is complete
        const int zo = zi - R;
        if (zo >= zb) {
            T* orow = dst + (int64_t)zo * plane;
#pragma unroll
            for (int vy = 0; vy < kVY; ++vy) {
                const int y = oy + vy;
                if (y >= j.Y) continue;
                T* o = orow + (int64_t)y * j.X + ox;
                T r4[kVX];
#pragma unroll
                for (int vx = 0; vx < kVX; ++vx) r4[vx] = finish<T, IACC>(acc[K - 1][vy][vx], j);
                if (j.vec_store && ox + kVX <= j.X) {
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
                        if (ox + vx < j.X) o[vx] = r4[vx];
                }
            }
        }
        // ---- advance the ring: slot c now belongs to output plane zi+1-c+r
#pragma unroll
        for (int c = K - 1; c > 0; --c)
#pragma unroll
            for (int vy = 0; vy < kVY; ++vy)
#pragma unroll
                for (int vx = 0; vx < kVX; ++vx) acc[c][vy][vx] = acc[c - 1][vy][vx];
#pragma unroll
        for (int vy = 0; vy < kVY; ++vy)
#pragma unroll
            for (int vx = 0; vx < kVX; ++vx) acc[0][vy][vx] = 0;
        __syncthreads();
    }
}

template <typename T, int K, bool IACC>
hipError_t launch_k(const FilterJob& j, hipStream_t s)
{
    const int tiles_x = (j.X + kTX - 1) / kTX, tiles_y = (j.Y + kTY - 1) / kTY;
    const int64_t ntiles = (int64_t)tiles_x * tiles_y;
    // z-slab depth: enough workgroups to fill 256 CUs several times over,
    // slabs deep enough to amortise the 2r halo planes.
    int64_t want_slabs = (2048 + ntiles - 1) / ntiles;
    int tz = (int)((j.Z + want_slabs - 1) / want_slabs);
    const int tz_min = 4 > 2 * K ? 4 : 2 * K;
    if (tz < tz_min) tz = tz_min;
    if (tz > 64) tz = 64;
    if (tz > j.Z) tz = j.Z;
    const int64_t slabs = (j.Z + tz - 1) / tz;
    const int64_t nb = ntiles * slabs;
    if (nb > 0x7fffffff) return hipErrorInvalidValue;
    using Acc = typename AccT<IACC>::type;
    const Acc* w;
    if constexpr (IACC) w = j.wi; else w = j.wf;
    hipLaunchKernelGGL((filter_valu_kernel<T, K, IACC>), dim3((unsigned)nb), dim3(kNT),
                       0, s, static_cast<const T*>(j.src), static_cast<T*>(j.dst), w,
                       j, tz, tiles_x, tiles_y, (uint32_t)nb);
    return hipGetLastError();
}

template <typename T, bool IACC>
hipError_t dispatch_k(const FilterJob& j, hipStream_t s)
{
    switch (j.k) {
    case 1: return launch_k<T, 1, IACC>(j, s);
    case 3: return launch_k<T, 3, IACC>(j, s);
    case 5: return launch_k<T, 5, IACC>(j, s);
    case 7: return launch_k<T, 7, IACC>(j, s);
    case 9: return launch_k<T, 9, IACC>(j, s);
    case 11: return launch_k<T, 11, IACC>(j, s);
    case 13: return launch_k<T, 13, IACC>(j, s);
    case 15: return launch_k<T, 15, IACC>(j, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_filter_valu(const FilterJob& j, hipStream_t s)
{
    switch (j.fmt) {
    case vktDataFormatUInt8:
        return j.int_acc ? dispatch_k<uint8_t, true>(j, s) : dispatch_k<uint8_t, false>(j, s);
    case vktDataFormatUInt16:
        return j.int_acc ? dispatch_k<uint16_t, true>(j, s) : dispatch_k<uint16_t, false>(j, s);
    case vktDataFormatFloat32:
        return dispatch_k<float, false>(j, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace vkt
