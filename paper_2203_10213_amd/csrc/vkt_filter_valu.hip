// vkt_filter_valu.hip -- ApplyFilter on the vector ALUs: FP32 fused
// multiply-add, or exact 24-bit integer multiply-add for integer-weight
// filters whose sums could leave the exactly representable FP32 range.
//
// Operation (paper Sec. 3.2 "Volume Manipulation"; benchmarked as a Gaussian
// blur of structured volumes in Sec. 4.3): for every output cell,
//   T(x,y,z) = sum_{a,b,c} w[a + k(b + k c)] * s(A(x+a-r), A(y+b-r), A(z+c-r)).
//
// Mapping to gfx950:
//  * A workgroup of 256 threads owns a 64 x 32 (x, y) output tile and marches
//    through a z-slab of output planes.  Each input plane of the slab, with an
//    r-wide halo in x and y, is gathered once (address mode applied to halo
//    coordinates only, through per-thread 32-bit in-plane offsets computed once
//    per tile) and staged in LDS as FP32 (or int32), double buffered; the
//    loads of the plane after next are in flight while a plane is computed.
//  * Input-stationary z ring: a thread owns 4 (x) x 2 (y) output columns and
//    keeps k partial sums per output, one for each output plane zi - c + r the
//    current input plane zi feeds.  A plane is read from LDS once per thread
//    (16-byte reads of its (4+k-1)-wide row windows) and feeds all k^3 taps.
//    After the plane, the ring's oldest entry is a finished output: it is
//    rounded, stored, and the ring advances.
//  * Weights are uniform: they are scalar operands of the multiply-adds,
//    loaded one group (a filter plane for k = 3, the rows (c, b), (c+1, b)
//    for k = 5, 7, else a filter row) at a time with explicit scalar loads
//    and one wait per group.  For k >= 5 the row windows stream through
//    registers one input row at a time.
//  * Single-volume launches number workgroups XCD-aware so tiles adjacent in
//    x/y at the same z share an XCD's L2 for their halo re-reads; batched
//    launches run persistent workgroups that take tile-slabs of many volumes
//    from a work queue.
#include "vkt_internal.h"

#include <type_traits>
#include <utility>

namespace vkt {
namespace {

// Filter rows loaded per scalar wait on the row-streaming path (k = 5, 7):
// two rows (of consecutive filter planes) measured 2 % faster than one on
// the 512^3 5^3 workload; three spill SGPRs at k = 7.
constexpr int kValuRowGroup = 2;
// Waves per SIMD the single-volume kernel is compiled for: the 5^3 FP32
// kernel fits 80 registers (six waves instead of five) with one spilled
// register, measured 3.6 % faster on the 512^3 workload; other sizes would
// spill a dozen registers and take what they need.
constexpr int valu_waves(int k, bool iacc) { return k == 5 && !iacc ? 6 : 1; }

constexpr int kBX = 16, kBY = 16, kNT = kBX * kBY;  // threads per workgroup
constexpr int kVX = 4, kVY = 2;                      // outputs per thread
constexpr int kTX = kBX * kVX, kTY = kBY * kVY;      // 64 x 32 tile
// (the batched form also has a 64 x 16 tile variant: one output row per
// thread, VY = 1)

template <int K, int VY = kVY>
struct Geo {
    static constexpr int R = (K - 1) / 2;
    static constexpr int HX = kTX + 2 * R;                // halo tile width
    static constexpr int HY = kBY * VY + 2 * R;           // halo tile height
    static constexpr int P = (HX + 3) & ~3;               // LDS row pitch (cells)
    static constexpr int NE = (HX * HY + kNT - 1) / kNT;  // halo cells per thread
    static constexpr int WX = kVX + K - 1;                // row window per thread
    static constexpr int NR = (WX + 3) / 4;               // 16-byte reads per row
    static constexpr int NROW = VY + K - 1;               // input rows per thread
    static constexpr int LDS_CELLS = HY * P;              // one plane buffer
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

// Weight rows are read with explicit scalar loads that wait for their data
// in the same statement.  The volatile statements keep their program order,
// so one weight group at a time is live in SGPRs: the loads are neither
// hoisted out of the z loop nor all issued at its top (which would spill
// SGPRs into VGPR lanes).  A load of N dwords may read up to N - 1 dwords
// past the last weight; weight buffers carry kWeightPad dwords of padding.
template <int N> struct SRow;
template <> struct SRow<4> { typedef uint32_t type __attribute__((ext_vector_type(4))); };
template <> struct SRow<8> { typedef uint32_t type __attribute__((ext_vector_type(8))); };
template <> struct SRow<16> { typedef uint32_t type __attribute__((ext_vector_type(16))); };

template <int N, typename Acc>
__device__ inline void load_weights(const Acc* p, Acc (&wv)[N])
{
    typename SRow<N>::type r;
    if constexpr (N == 4)
        asm volatile("s_load_dwordx4 %0, %1, 0x0\n\ts_waitcnt lgkmcnt(0)" : "=&s"(r) : "s"(p));
    else if constexpr (N == 8)
        asm volatile("s_load_dwordx8 %0, %1, 0x0\n\ts_waitcnt lgkmcnt(0)" : "=&s"(r) : "s"(p));
    else
        asm volatile("s_load_dwordx16 %0, %1, 0x0\n\ts_waitcnt lgkmcnt(0)" : "=&s"(r) : "s"(p));
#pragma unroll
    for (int q = 0; q < N; ++q) {
        const uint32_t u = r[q];
        if constexpr (std::is_same<Acc, float>::value) wv[q] = __uint_as_float(u);
        else wv[q] = (Acc)u;
    }
}

// G filter rows of N weights, rows `stride` weights apart, issued as G
// scalar loads followed by one wait (one wait per group of rows instead of
// one per row).
template <int N, int G, typename Acc>
__device__ inline void load_weight_rows(const Acc* p, int stride, Acc (&wv)[G][N])
{
    static_assert(N == 8 && G >= 1 && G <= 3, "rows of 8 dwords, up to 3 per group");
    typename SRow<8>::type r0, r1, r2;
    const Acc* p1 = p + stride;
    const Acc* p2 = p + 2 * stride;
    if constexpr (G == 1)
        asm volatile("s_load_dwordx8 %0, %1, 0x0\n\ts_waitcnt lgkmcnt(0)" : "=&s"(r0) : "s"(p));
    else if constexpr (G == 2)
        asm volatile("s_load_dwordx8 %0, %2, 0x0\n\ts_load_dwordx8 %1, %3, 0x0\n\t"
                     "s_waitcnt lgkmcnt(0)"
                     : "=&s"(r0), "=&s"(r1) : "s"(p), "s"(p1));
    else
        asm volatile("s_load_dwordx8 %0, %3, 0x0\n\ts_load_dwordx8 %1, %4, 0x0\n\t"
                     "s_load_dwordx8 %2, %5, 0x0\n\ts_waitcnt lgkmcnt(0)"
                     : "=&s"(r0), "=&s"(r1), "=&s"(r2) : "s"(p), "s"(p1), "s"(p2));
#pragma unroll
    for (int q = 0; q < N; ++q) {
        const uint32_t u[3] = {r0[q], G > 1 ? r1[q] : 0u, G > 2 ? r2[q] : 0u};
#pragma unroll
        for (int g = 0; g < G; ++g) {
            if constexpr (std::is_same<Acc, float>::value) wv[g][q] = __uint_as_float(u[g]);
            else wv[g][q] = (Acc)u[g];
        }
    }
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

// Dwords of a scalar load covering n weights.
constexpr int sload_width(int n) { return n <= 4 ? 4 : n <= 8 ? 8 : 16; }

// Raw buffer loads: SGPR resource (base, size) + 32-bit VGPR byte offset.
// An offset at or beyond the resource size reads 0 (used for border cells).
constexpr uint32_t kRsrcWord3 = 0x00020000u;   // gfx9-family raw buffer
constexpr uint32_t kOutside = 0x80000000u;     // byte offset that reads 0

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

template <bool IACC> struct AccT { using type = float; };
template <> struct AccT<true> { using type = int32_t; };

__device__ inline float mac(float w, float v, float acc) { return fmaf(w, v, acc); }
__device__ inline int32_t mac(int32_t w, int32_t v, int32_t acc)
{
    return __mul24(w, v) + acc;  // |w| < 2^23, cells < 2^16: exact
}

__device__ inline uint32_t udiv(uint32_t n, UDiv d)
{
    const uint32_t t = __umulhi(d.m, n);
    return (t + ((n - t) >> d.sh1)) >> d.sh2;
}

// Stored value of one finished output.
template <typename T, typename Acc>
__device__ inline T finish(Acc acc, const VolDesc& a)
{
    if constexpr (std::is_same<T, float>::value) {
        return a.epi == kEpiFloatDiv ? (float)acc * a.inv_D : (float)acc;
    } else {
        constexpr int kMax = std::is_same<T, uint8_t>::value ? 255 : 65535;
        if (a.epi == kEpiIntDiv) {
            // acc is an exact integer (int32, or float below 2^24)
            const int32_t t = (int32_t)acc;
            if (t < 0) return (T)0;
            const uint32_t q = udiv(2u * (uint32_t)t + (uint32_t)a.D, a.div2D);
            return (T)(q > (uint32_t)kMax ? (uint32_t)kMax : q);
        }
        const float q = floorf((float)acc + 0.5f);
        return (T)fminf(fmaxf(q, 0.f), (float)kMax);
    }
}

// One tile-slab: output tile `tile` of z-slab `slab` of volume a.
template <typename T, int K, bool IACC, int VY = kVY>
__device__ void valu_tile(const VolDesc& a, const typename AccT<IACC>::type* __restrict__ w,
                          int tile, int slab, typename AccT<IACC>::type* lds)
{
    using G = Geo<K, VY>;
    constexpr int kVY = VY, kTY = kBY * VY;
    using Acc = typename AccT<IACC>::type;
    constexpr int R = G::R;
    const T* __restrict__ src = static_cast<const T*>(a.src);
    T* __restrict__ dst = static_cast<T*>(a.dst);

    const int t = threadIdx.x, tx = t % kBX, ty = t / kBX;
    const int x0 = a.rx0 + (tile % a.tiles_x) * kTX, y0 = a.ry0 + (tile / a.tiles_x) * kTY;
    const int zb = a.rz0 + slab * a.tz, ze = min(zb + a.tz, a.rz1);
    const int64_t plane = (int64_t)a.X * a.Y;

    // Halo gather: the same (x, y) cells for every plane of the slab.
    uint32_t goff[G::NE];   // in-plane source byte offset (kOutside: zero cell)
    int32_t loff[G::NE];    // LDS slot
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
    Acc stage[G::NE];
    auto gather = [&](int zi) {
        const int gz = addr_map(zi, a.Z, a.mode);  // -1 only for border: a zero plane
        const char* base = reinterpret_cast<const char*>(src) +
                           (gz < 0 ? 0 : (int64_t)gz * plane_bytes);
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<char*>(base), (short)0, gz < 0 ? 0 : plane_bytes, (int)kRsrcWord3);
#pragma unroll
        for (int i = 0; i < G::NE; ++i) stage[i] = (Acc)buf_load<T>(rs, goff[i]);
    };
    auto put = [&](Acc* buf) {
#pragma unroll
        for (int i = 0; i < G::NE; ++i) buf[loff[i]] = stage[i];
    };

    Acc acc[K][kVY][kVX];
#pragma unroll
    for (int c = 0; c < K; ++c)
#pragma unroll
        for (int vy = 0; vy < kVY; ++vy)
#pragma unroll
            for (int vx = 0; vx < kVX; ++vx) acc[c][vy][vx] = 0;

    const int zi_beg = zb - R, zi_end = ze + R;  // input planes [beg, end)
    // planes zi_beg and zi_beg + 1 in flight before the loop; iteration zi
    // stages plane zi + 1 (loaded during iteration zi - 1) and issues the
    // loads of plane zi + 2, so a load has a whole plane of taps to arrive
    gather(zi_beg);
    put(lds);
    if (zi_beg + 1 < zi_end) gather(zi_beg + 1);
    __syncthreads();

    const int ox = x0 + kVX * tx, oy = y0 + kVY * ty;
    const bool vec = a.vec_ok && ox + kVX <= a.rx1;
    for (int zi = zi_beg; zi < zi_end; ++zi) {
        const int cur = (zi - zi_beg) & 1;
        if (zi + 1 < zi_end) put(lds + (cur ^ 1) * G::LDS_CELLS);
        if (zi + 2 < zi_end) gather(zi + 2);

        const Acc* buf = lds + cur * G::LDS_CELLS + (kVY * ty) * G::P + kVX * tx;
        // ring slot c feeds output plane zi - c + r; slots outside the slab's
        // output planes [zb, ze) are never stored, so their taps are skipped
        const int c_lo = max(0, zi + R - ze + 1), c_hi = min(K - 1, zi + R - zb);
        using V4 = typename std::conditional<IACC, int4, float4>::type;
        if constexpr (K <= 3) {
            // all (2 + k - 1) row windows in registers, then the taps of one
            // filter plane c at a time
            Acc v[G::NROW][G::NR * 4];
#pragma unroll
            for (int jr = 0; jr < G::NROW; ++jr)
#pragma unroll
                for (int q = 0; q < G::NR; ++q) {
                    const V4 u = *reinterpret_cast<const V4*>(buf + jr * G::P + 4 * q);
                    v[jr][4 * q + 0] = u.x;
                    v[jr][4 * q + 1] = u.y;
                    v[jr][4 * q + 2] = u.z;
                    v[jr][4 * q + 3] = u.w;
                }
#pragma unroll
            for (int c = 0; c < K; ++c) {
                if (c < c_lo || c > c_hi) continue;
                constexpr int NW = sload_width(K * K);
                Acc wv[NW];
                load_weights<NW>(w + c * K * K, wv);
#pragma unroll
                for (int b = 0; b < K; ++b)
#pragma unroll
                    for (int aa = 0; aa < K; ++aa)
#pragma unroll
                        for (int vy = 0; vy < kVY; ++vy)
#pragma unroll
                            for (int vx = 0; vx < kVX; ++vx)
                                acc[c][vy][vx] = mac(wv[b * K + aa], v[b + vy][vx + aa],
                                                     acc[c][vy][vx]);
            }
        } else {
            // stream the row windows; filter rows are loaded one (or, for
            // k <= 7, a group of planes') at a time
            constexpr int kRowGroup = K <= 7 ? kValuRowGroup : 1;
#pragma unroll 1
            for (int jr = 0; jr < G::NROW; ++jr) {
                Acc v[G::NR * 4];
#pragma unroll
                for (int q = 0; q < G::NR; ++q) {
                    const V4 u = *reinterpret_cast<const V4*>(buf + jr * G::P + 4 * q);
                    v[4 * q + 0] = u.x;
                    v[4 * q + 1] = u.y;
                    v[4 * q + 2] = u.z;
                    v[4 * q + 3] = u.w;
                }
#pragma unroll
                for (int vy = 0; vy < kVY; ++vy) {
                    const int b = jr - vy;
                    if (b < 0 || b >= K) continue;
                    if constexpr (kRowGroup > 1) {
                        // filter rows (c, b) of kRowGroup consecutive planes c
                        // per scalar wait
                        constexpr int NGRP = (K + kRowGroup - 1) / kRowGroup;
                        static_for<NGRP>([&](auto gi) {
                            constexpr int c0 = decltype(gi)::value * kRowGroup;
                            constexpr int GN = K - c0 < kRowGroup ? K - c0 : kRowGroup;
                            if (c0 + GN - 1 < c_lo || c0 > c_hi) return;
                            Acc wv[GN][8];
                            load_weight_rows<8, GN>(w + (c0 * K + b) * K, K * K, wv);
#pragma unroll
                            for (int g = 0; g < GN; ++g) {
                                const int c = c0 + g;
                                if (c < c_lo || c > c_hi) continue;
#pragma unroll
                                for (int aa = 0; aa < K; ++aa)
#pragma unroll
                                    for (int vx = 0; vx < kVX; ++vx)
                                        acc[c][vy][vx] = mac(wv[g][aa], v[vx + aa], acc[c][vy][vx]);
                            }
                        });
                    } else {
#pragma unroll
                    for (int c = 0; c < K; ++c) {
                        if (c < c_lo || c > c_hi) continue;
                        constexpr int NW = sload_width(K);
                        Acc wv[NW];
                        load_weights<NW>(w + (c * K + b) * K, wv);
#pragma unroll
                        for (int aa = 0; aa < K; ++aa)
#pragma unroll
                            for (int vx = 0; vx < kVX; ++vx)
                                acc[c][vy][vx] = mac(wv[aa], v[vx + aa], acc[c][vy][vx]);
                    }
                    }
                }
            }
        }

        // ---- the ring's oldest entry is output plane zo = zi - r
        const int zo = zi - R;
        if (zo >= zb) {
            T* orow = dst + (int64_t)zo * plane;
#pragma unroll
            for (int vy = 0; vy < kVY; ++vy) {
                const int y = oy + vy;
                if (y >= a.ry1) continue;
                T* o = orow + (int64_t)y * a.X + ox;
                T r4[kVX];
#pragma unroll
                for (int vx = 0; vx < kVX; ++vx) r4[vx] = finish<T>(acc[K - 1][vy][vx], a);
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
__global__ __launch_bounds__(kNT) __attribute__((amdgpu_waves_per_eu(valu_waves(K, IACC))))
void filter_valu_kernel(
    VolDesc a, const typename AccT<IACC>::type* __restrict__ w, uint32_t nblocks)
{
    using Acc = typename AccT<IACC>::type;
    __shared__ __align__(16) Acc lds[2 * Geo<K>::LDS_CELLS];
    const uint32_t lid = xcd_remap(blockIdx.x, nblocks);
    const uint32_t ntiles = (uint32_t)a.tiles_x * (uint32_t)a.tiles_y;
    valu_tile<T, K, IACC>(a, w, (int)(lid % ntiles), (int)(lid / ntiles), lds);
}

// Persistent workgroups: take items (volume, tile-slab) from the queue until
// it is empty; the last workgroup to finish resets the queue counters.
template <typename T, int K, bool IACC, int VY>
__global__ __launch_bounds__(kNT) void filter_valu_batched_kernel(BatchArgs b)
{
    using Acc = typename AccT<IACC>::type;
    __shared__ __align__(16) Acc lds[2 * Geo<K, VY>::LDS_CELLS];
    __shared__ uint32_t s_item;
    const Acc* pool;
    if constexpr (IACC) pool = b.wipool; else pool = b.wpool;
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(&b.counters[0], 1u);
        __syncthreads();
        // the item index is the same in every lane: keep it (and the work item
        // and volume descriptor it selects) in scalar registers
        const uint32_t it = (uint32_t)__builtin_amdgcn_readfirstlane((int)s_item);
        __syncthreads();
        if (it >= b.nitems) break;
        const WorkItem wi = uniform_load(&b.items[it]);
        const VolDesc a = uniform_load(&b.vols[wi.vol]);
        const uint32_t ntiles = (uint32_t)a.tiles_x * (uint32_t)a.tiles_y;
        valu_tile<T, K, IACC, VY>(a, pool + a.woff, (int)(wi.lid % ntiles),
                                  (int)(wi.lid / ntiles), lds);
    }
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(&b.counters[1], 1u) == gridDim.x - 1) {
            atomicExch(&b.counters[0], 0u);
            atomicExch(&b.counters[1], 0u);
        }
    }
}

// Output regions up to this many cells (k <= 3: the 27 weights stay in
// SGPRs) take the direct kernel, in workgroups of kDirectBX x kDirectBY.
constexpr int64_t kDirectMaxCells = int64_t(1) << 19;
constexpr int kDirectBX = 64, kDirectBY = kNT / kDirectBX;

// Small output regions: one thread per output cell reading its k^3 taps
// straight from memory (the whole source is cache resident at these sizes),
// with no LDS staging and no barriers, so a 64^3 volume is 1024 workgroups in
// one wave of the device instead of a few dozen tile-slabs.  Workgroups of
// 64 x 4 threads cover 64 x 4 outputs of one plane (grid: x runs, y runs,
// planes), so a thread finds its cell without divisions.  Taps are summed
// in the tiled kernel's order (filter plane, row, column).
template <typename T, int K, bool IACC>
__global__ __launch_bounds__(kNT) void filter_direct_kernel(
    VolDesc a, const typename AccT<IACC>::type* __restrict__ w)
{
    using Acc = typename AccT<IACC>::type;
    constexpr int R = (K - 1) / 2;
    const int x = a.rx0 + (int)blockIdx.x * kDirectBX + (int)threadIdx.x;
    const int y = a.ry0 + (int)blockIdx.y * kDirectBY + (int)threadIdx.y;
    const int z = a.rz0 + (int)blockIdx.z;
    if (x >= a.rx1 || y >= a.ry1) return;
    int xs[K], ys[K], zs[K];  // coordinates through the address mode; -1: zero
#pragma unroll
    for (int t = 0; t < K; ++t) {
        xs[t] = addr_map((int64_t)x + t - R, a.X, a.mode);
        ys[t] = addr_map((int64_t)y + t - R, a.Y, a.mode);
        zs[t] = addr_map((int64_t)z + t - R, a.Z, a.mode);
    }
    const T* __restrict__ src = static_cast<const T*>(a.src);
    Acc acc = 0;
#pragma unroll
    for (int c = 0; c < K; ++c)
#pragma unroll
        for (int b = 0; b < K; ++b) {
            // cells outside under border read as zero: the load goes to a
            // cell inside the volume and its value is replaced
            const bool row_in = zs[c] >= 0 && ys[b] >= 0;
            const T* row = src + ((int64_t)max(zs[c], 0) * a.Y + max(ys[b], 0)) * a.X;
#pragma unroll
            for (int aa = 0; aa < K; ++aa) {
                const Acc cell = (Acc)row[max(xs[aa], 0)];
                const Acc v = (row_in && xs[aa] >= 0) ? cell : (Acc)0;
                acc = mac(w[(c * K + b) * K + aa], v, acc);
            }
        }
    T* __restrict__ dst = static_cast<T*>(a.dst);
    dst[((int64_t)z * a.Y + y) * a.X + x] = finish<T>(acc, a);
}


template <typename T, int K, bool IACC>
hipError_t launch_k(const FilterJob& j, hipStream_t s)
{
    const ClassGeom g = valu_geom(K);
    using Acc = typename AccT<IACC>::type;
    const Acc* w;
    if constexpr (IACC) w = j.wi; else w = j.wf;
    {
        const int64_t cells =
            (int64_t)(j.roi[3] - j.roi[0]) * (j.roi[4] - j.roi[1]) * (j.roi[5] - j.roi[2]);
        if constexpr (K <= 3) {
            const int RY = j.roi[4] - j.roi[1], RZ = j.roi[5] - j.roi[2];
            const int gy = (RY + kDirectBY - 1) / kDirectBY;
            if (cells <= kDirectMaxCells && gy <= 65535 && RZ <= 65535) {
                const VolDesc a = make_desc(j, 1, g);
                const int gx = (j.roi[3] - j.roi[0] + kDirectBX - 1) / kDirectBX;
                hipLaunchKernelGGL((filter_direct_kernel<T, K, IACC>),
                                   dim3((unsigned)gx, (unsigned)gy, (unsigned)RZ),
                                   dim3(kDirectBX, kDirectBY), 0, s, a, w);
                return hipGetLastError();
            }
        }
    }
    // the output region's tiles and z extent (the whole volume unless a range)
    const int RX = j.roi[3] - j.roi[0], RY = j.roi[4] - j.roi[1], RZ = j.roi[5] - j.roi[2];
    const int64_t ntiles = (int64_t)((RX + g.tx - 1) / g.tx) * ((RY + g.ty - 1) / g.ty);
    const void* fn = (const void*)&filter_valu_kernel<T, K, IACC>;
    const int tz = plan_tz(ntiles, RZ, K, 1, 128, resident_wgs(fn), 1);
    const VolDesc a = make_desc(j, tz, g);
    const int64_t nb = ntiles * ((RZ + tz - 1) / tz);
    if (nb > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL((filter_valu_kernel<T, K, IACC>), dim3((unsigned)nb), dim3(kNT), 0, s,
                       a, w, (uint32_t)nb);
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

template <typename T, bool IACC, int VY>
const void* batched_vy(int k)
{
    switch (k) {
    case 1: return (const void*)&filter_valu_batched_kernel<T, 1, IACC, VY>;
    case 3: return (const void*)&filter_valu_batched_kernel<T, 3, IACC, VY>;
    case 5: return (const void*)&filter_valu_batched_kernel<T, 5, IACC, VY>;
    case 7: return (const void*)&filter_valu_batched_kernel<T, 7, IACC, VY>;
    case 9: return (const void*)&filter_valu_batched_kernel<T, 9, IACC, VY>;
    case 11: return (const void*)&filter_valu_batched_kernel<T, 11, IACC, VY>;
    case 13: return (const void*)&filter_valu_batched_kernel<T, 13, IACC, VY>;
    case 15: return (const void*)&filter_valu_batched_kernel<T, 15, IACC, VY>;
    }
    return nullptr;
}

// tile variant 0: 64 x 32 (two output rows per thread); 1: 64 x 16
template <typename T, bool IACC>
const void* batched_k(int k, int variant)
{
    return variant ? batched_vy<T, IACC, 1>(k) : batched_vy<T, IACC, kVY>(k);
}

}  // namespace

ClassGeom valu_geom(int k, int variant)
{
    ClassGeom g;
    g.tx = kTX;
    g.ty = variant ? kBY : kTY;
    g.tz_min = 4 > 2 * k ? 4 : 2 * k;
    return g;
}

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

const void* valu_batched_kernel(vktDataFormat f, int k, bool int_acc, int variant)
{
    switch (f) {
    case vktDataFormatUInt8:
        return int_acc ? batched_k<uint8_t, true>(k, variant)
                       : batched_k<uint8_t, false>(k, variant);
    case vktDataFormatUInt16:
        return int_acc ? batched_k<uint16_t, true>(k, variant)
                       : batched_k<uint16_t, false>(k, variant);
    case vktDataFormatFloat32:
        return int_acc ? nullptr : batched_k<float, false>(k, variant);
    }
    return nullptr;
}

}  // namespace vkt
