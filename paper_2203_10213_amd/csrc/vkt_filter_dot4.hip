// vkt_filter_dot4.hip -- ApplyFilter for uint8 volumes with small integer
// filters, on the vector ALUs with 4-way 8-bit dot products (v_dot4).
//
// Operation (paper Sec. 3.2 "Volume Manipulation"; benchmarked as a blur of
// structured volumes in Sec. 4.3): for every output cell
//   T(x,y,z) = sum_{a,b,c} w[a + k(b + k c)] * s(A(x+a-r), A(y+b-r), A(z+c-r)),
//   out      = clamp(floor((2T + D) / 2D), 0, 255).
//
// Eligible jobs (decided on the host): uint8 cells, integer weights all in
// [0, 255] (unsigned dot products) or all in [-128, 127] (signed: every cell
// enters as s - 128 and the constant 128 * sum(w) is folded into the
// epilogue), k in {3, 5, 7}, sum |w| <= 2048, 1 <= D <= 2^19, rows of a
// multiple of 4 cells, 4-byte aligned buffers.
//
// Mapping to gfx950:
//  * A workgroup of 4 waves owns a 256 x 4VY (x, y) output tile and marches
//    through a z-slab.  A lane owns 4 consecutive x outputs (one dword of an
//    output row) in VY rows.
//  * Each input plane of the slab, with its halo, is staged in LDS as raw
//    bytes, double buffered: rows of 66 dwords (one halo dword on either
//    side).  Dwords inside the volume are single 32-bit loads; only dwords
//    past an x face go through the address mode byte by byte.
//  * Per input row a lane reads the dword left of, at and right of its own
//    and forms the 4-byte windows at every tap offset with v_alignbyte.
//  * Each filter row (c, b) is packed into ceil(k/4) dwords of 8-bit weights
//    (zero past k): one v_dot4 adds 4 taps of one output, a filter row costs
//    1 (k = 3) or 2 (k = 5, 7) dot products per output.
//  * Input-stationary z ring of k partial sums per output; the z loop is
//    unrolled by k so the ring slots are fixed registers.
//  * Epilogue in FP32: T/D + 1/2 is a multiple of 1/(2D), so
//    floor(T/D + 1/2) = round-to-nearest(T * (1/D) + 1/(4D)) whenever the
//    FMA's rounding error stays below 1/(4D), which the eligibility bounds
//    guarantee (3 * 2^-24 * (256 sum|w| + D) < 1/4).  v_cvt_pk_u8_f32 does
//    the rounding, the saturation to [0, 255] and the packing of four
//    outputs into one dword store.
#include "vkt_internal.h"

#include <type_traits>
#include <utility>

namespace vkt {
namespace {

constexpr int kNT = 256, kWaves = 4, kLanes = 64;
constexpr int kTX = 4 * kLanes;  // output cells per tile row

// VYO: output rows per lane of a tile variant of the batched form (0: the
// default below; the other variant takes half as many rows)
template <int K, int VYO = 0>
struct Geo4 {
    static constexpr int R = (K - 1) / 2;
    static constexpr int VY_DEFAULT = K <= 3 ? 4 : 2;
    static constexpr int VY = VYO ? VYO : VY_DEFAULT;   // output rows per lane
    static constexpr int TY = kWaves * VY;              // tile rows
    static constexpr int HY = TY + 2 * R;               // staged rows per plane
    static constexpr int WD = kLanes + 2;               // dwords per staged row
    static constexpr int PLANE = HY * WD;               // dwords per staged plane
    static constexpr int PLANE_BUF = PLANE + 4;         // + a dummy dword (padded)
    static constexpr int NH = (K + 3) / 4;              // weight dwords per filter row
    static constexpr int NROW = VY + K - 1;             // input rows per lane
    static constexpr int WAVES = K <= 3 ? 4 : K <= 5 ? 3 : 2;  // occupancy target per SIMD
    static_assert(R <= 4, "one halo dword per side");
};

constexpr uint32_t kRsrcWord3 = 0x00020000u;  // gfx9-family raw buffer
constexpr uint32_t kOutside = 0x80000000u;    // byte offset that reads 0

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

__device__ inline uint32_t xcd_remap(uint32_t b, uint32_t n)
{
    const uint32_t q = n / 8, rem = n % 8, xcd = b % 8, idx = b / 8;
    return xcd < rem ? xcd * (q + 1) + idx : rem * (q + 1) + (xcd - rem) * q + idx;
}

template <typename F, int... I>
__device__ inline void static_for_impl(F& f, std::integer_sequence<int, I...>)
{
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ inline void static_for(F&& f)
{
    static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// Bytes o .. o+3 of a lane's 12-byte neighbourhood (L: x0-4.., C: x0.., R:
// x0+4..) as one dword, o in [-4, 7].  For o > 4 only the low bytes are
// meaningful (the matching weights are zero).
template <int O>
__device__ inline uint32_t window(uint32_t L, uint32_t C, uint32_t R)
{
    if constexpr (O == -4) return L;
    else if constexpr (O < 0) return __builtin_amdgcn_alignbyte(C, L, 4 + O);
    else if constexpr (O == 0) return C;
    else if constexpr (O < 4) return __builtin_amdgcn_alignbyte(R, C, O);
    else if constexpr (O == 4) return R;
    else return __builtin_amdgcn_alignbyte(R, R, O - 4);
}

template <bool SG>
__device__ inline int32_t dot4(uint32_t a, uint32_t w, int32_t acc)
{
    if constexpr (SG) return __builtin_amdgcn_sdot4((int)a, (int)w, acc, false);
    else return (int32_t)__builtin_amdgcn_udot4(a, w, (uint32_t)acc, false);
}

// One filter plane's packed weight rows (k rows x NH dwords <= 14 dwords) in
// SGPRs: one explicit 16-dword scalar load that waits for its data, so that
// only one plane's weights are live at a time.  Reads up to 2 dwords past the
// last filter plane; weight buffers carry kWeightPad dwords of padding.
__device__ inline void load_plane_weights(const uint32_t* p, uint32_t (&wv)[16])
{
    typedef uint32_t v16 __attribute__((ext_vector_type(16)));
    v16 r;
    asm volatile("s_load_dwordx16 %0, %1, 0x0\n\ts_waitcnt lgkmcnt(0)" : "=&s"(r) : "s"(p));
#pragma unroll
    for (int q = 0; q < 16; ++q) wv[q] = r[q];
}

// Orders the computation of 8 partial sums before every later volatile
// statement (an empty statement that claims to read and write them).
__device__ inline void pin8(int32_t (&v)[2][4])
{
    asm volatile("" : "+v"(v[0][0]), "+v"(v[0][1]), "+v"(v[0][2]), "+v"(v[0][3]),
                      "+v"(v[1][0]), "+v"(v[1][1]), "+v"(v[1][2]), "+v"(v[1][3]));
}
__device__ inline void pin8(int32_t (&v)[1][4])
{
    asm volatile("" : "+v"(v[0][0]), "+v"(v[0][1]), "+v"(v[0][2]), "+v"(v[0][3]));
}
template <int N>
__device__ inline void pin8(int32_t (&)[N][4])
{
    static_assert(N == 1 || N == 2, "rows per lane with scalar weight groups");
}

// One tile-slab: output tile `tile` of z-slab `slab` of volume a.
template <int K, bool SG, int VYO = 0>
__device__ void dot4_tile(const VolDesc& a, const uint32_t* __restrict__ wq, int tile,
                          int slab, uint32_t* lds)
{
    using G = Geo4<K, VYO>;
    constexpr int R = G::R, VY = G::VY, NH = G::NH;
    const uint8_t* __restrict__ src = static_cast<const uint8_t*>(a.src);
    uint8_t* __restrict__ dst = static_cast<uint8_t*>(a.dst);

    const int t = threadIdx.x, lane = t % kLanes, wave = t / kLanes;
    const int x0 = a.rx0 + (tile % a.tiles_x) * kTX, y0 = a.ry0 + (tile / a.tiles_x) * G::TY;
    const int zb = a.rz0 + slab * a.tz, ze = min(zb + a.tz, a.rz1);
    const int64_t plane = (int64_t)a.X * a.Y;

    // Staged dwords, the same (x, y) for every plane of the slab.  Interior
    // dwords (d = 1 .. 64 of a staged row) go to lane d - 1 of wave hy mod 4;
    // the two halo dwords of each row (d = 0 and the last one needed) to
    // threads 0 .. 2 HY - 1.  A dword is loaded whole, except the one just
    // past either x face of the volume, whose four bytes go through the
    // address mode.  Interior dwords at or past the right face are not
    // staged (they feed no stored output); halo slots of threads with no row
    // write a dummy LDS dword past the plane.
    constexpr int NI = (G::HY + kWaves - 1) / kWaves;  // interior slots per thread
    const int wv_u = __builtin_amdgcn_readfirstlane(wave);  // wave-uniform copy
    // interior slot i: row hy = wave + 4 i, a wave-uniform byte offset of the
    // staged row's first interior dword (SGPR) plus 4 * lane (VGPR)
    uint32_t srow[NI];
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        const int hy = wv_u + kWaves * i;
        const int gy = hy < G::HY ? addr_map((int64_t)y0 - R + hy, a.Y, a.mode) : -1;
        srow[i] = gy < 0 ? kOutside : (uint32_t)gy * (uint32_t)a.X + (uint32_t)x0;
    }
    const uint32_t vlane = 4u * (uint32_t)lane;
    const bool xin = x0 + 4 * lane + 4 <= a.X;               // dword inside the volume
    uint32_t* const lrow = lds + wave * G::WD + 1 + lane;    // slot 0's LDS dword (buffer 0)
    uint32_t goff[NI + 1];  // [NI]: byte offset of the halo dword (face dwords: of the row)
    int32_t loff[NI + 1];   // [NI]: its LDS dword
    // halo slot: row t / 2, left (even t) or right (odd t) neighbour dword
    bool face;
    int fside;
    {
        const int hy = t / 2, right = t % 2;
        const bool live = t < 2 * G::HY;
        const int gy = live ? addr_map((int64_t)y0 - R + hy, a.Y, a.mode) : -1;
        const int xr = min(x0 + kTX, a.X);  // first cell right of the staged part
        const int xb = right ? xr : x0 - 4;
        face = gy >= 0 && (right ? xr == a.X : x0 == 0);  // rows outside read zero whole
        fside = right;
        const uint32_t row = gy < 0 ? 0u : (uint32_t)gy * (uint32_t)a.X;
        goff[NI] = gy < 0 ? kOutside : (face ? row : row + (uint32_t)xb);
        loff[NI] = live ? hy * G::WD + (xb - (x0 - 4)) / 4 : G::PLANE;
    }
    // byte offsets (relative to the row) of the 4 cells past either x face
    // under the address mode (X >= 4); kOutside reads zero
    uint32_t fx[2][4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        switch (a.mode) {
        case vktAddressModeClamp: fx[0][q] = 0; fx[1][q] = a.X - 1; break;
        case vktAddressModeWrap: fx[0][q] = a.X - 4 + q; fx[1][q] = q; break;
        case vktAddressModeMirror: fx[0][q] = 3 - q; fx[1][q] = a.X - 1 - q; break;
        default: fx[0][q] = kOutside; fx[1][q] = kOutside; break;
        }
    }

    const int32_t plane_bytes = (int32_t)plane;  // < 2^31 (host check)
    uint32_t stage[NI + 1];
    auto gather = [&](int zi) {
        const int gz = addr_map(zi, a.Z, a.mode);  // -1 only for border: a zero plane
        const char* base = reinterpret_cast<const char*>(src) +
                           (gz < 0 ? 0 : (int64_t)gz * plane_bytes);
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<char*>(base), (short)0, gz < 0 ? 0 : plane_bytes, (int)kRsrcWord3);
#pragma unroll
        for (int i = 0; i < NI; ++i)
            stage[i] = __builtin_amdgcn_raw_buffer_load_b32(rs, (int)vlane, (int)srow[i], 0);
        stage[NI] = __builtin_amdgcn_raw_buffer_load_b32(rs, (int)goff[NI], 0, 0);
        if (face) {
            uint32_t v = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const uint32_t off = goff[NI] + (fside ? fx[1][q] : fx[0][q]);
                v |= (uint32_t)__builtin_amdgcn_raw_buffer_load_b8(rs, (int)off, 0, 0) << (8 * q);
            }
            stage[NI] = v;
        }
    };
    auto put = [&](int b) {
        if (xin) {
#pragma unroll
            for (int i = 0; i < NI; ++i)
                if (wv_u + kWaves * i < G::HY) lrow[b * G::PLANE_BUF + i * kWaves * G::WD] = stage[i];
        }
        lds[b * G::PLANE_BUF + loff[NI]] = stage[NI];
    };

    int32_t acc[K][VY][4];
#pragma unroll
    for (int c = 0; c < K; ++c)
#pragma unroll
        for (int vy = 0; vy < VY; ++vy)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[c][vy][j] = 0;

    const int zi_beg = zb - R;
    const int nz = ze - zb;           // output planes of the slab
    const int P = nz + 2 * R;         // input planes of the slab
    // planes 0 and 1 in flight before the first step; step p stages plane
    // p + 1 (loaded during step p - 1) and issues the loads of plane p + 2,
    // so a load has a whole step of taps to arrive
    gather(zi_beg);
    put(0);
    if (P > 1) gather(zi_beg + 1);
    __syncthreads();

    const int ox = x0 + 4 * lane;
    const bool x_ok = ox < a.rx1;  // rx1 is a multiple of 4
    const float inv_D = a.inv_D, bias = a.bias;

    // input plane p of the slab at ring position U = p mod k
    auto step = [&](int p, auto uc) {
        constexpr int U = decltype(uc)::value;
        if (p + 1 < P) put((p + 1) & 1);
        if (p + 2 < P) gather(zi_beg + p + 2);
        // the dot products at raised wave priority: the issue arbiter prefers
        // waves in this phase over waves staging or storing (512^3 3^3:
        // 0.097 -> 0.090 ms; the FP32 vector kernel gained nothing from it)
        __builtin_amdgcn_s_setprio(1);
        const uint32_t* buf = lds + (p & 1) * G::PLANE_BUF + (wave * VY) * G::WD + lane;

        if constexpr (K <= 3) {
            // stream the input rows: the 4 windows of row jr feed every
            // (output row vy, filter row b = jr - vy, filter plane c)
#pragma unroll
            for (int jr = 0; jr < G::NROW; ++jr) {
                uint32_t L = buf[jr * G::WD], C = buf[jr * G::WD + 1], Rr = buf[jr * G::WD + 2];
                if constexpr (SG) {
                    L ^= 0x80808080u;
                    C ^= 0x80808080u;
                    Rr ^= 0x80808080u;
                }
                uint32_t win[4];
                static_for<4>([&](auto qc) {
                    constexpr int j = decltype(qc)::value;
                    win[j] = window<j - R>(L, C, Rr);
                });
                static_for<K>([&](auto cc) {
                    constexpr int c = decltype(cc)::value;
                    constexpr int slot = ((U - c) % K + K) % K;
                    // filter plane c feeds output plane p - c of the slab:
                    // skip planes outside it (never stored)
                    if (p - c < 0 || p - c >= nz) return;
#pragma unroll
                    for (int vy = 0; vy < VY; ++vy) {
                        const int b = jr - vy;
                        if (b < 0 || b >= K) continue;
                        const uint32_t wrow = wq[(c * K + b) * NH];
#pragma unroll
                        for (int j = 0; j < 4; ++j)
                            acc[slot][vy][j] = dot4<SG>(win[j], wrow, acc[slot][vy][j]);
                    }
                });
            }
        } else {
            // the 4 NH windows of every input row this lane needs, then one
            // filter plane c (weights in SGPRs) at a time
            uint32_t win[G::NROW][4 * NH];
#pragma unroll
            for (int jr = 0; jr < G::NROW; ++jr) {
                uint32_t L = buf[jr * G::WD], C = buf[jr * G::WD + 1], Rr = buf[jr * G::WD + 2];
                if constexpr (SG) {
                    L ^= 0x80808080u;
                    C ^= 0x80808080u;
                    Rr ^= 0x80808080u;
                }
                static_for<4 * NH>([&](auto qc) {
                    constexpr int q = decltype(qc)::value;
                    constexpr int h = q / 4, j = q % 4;
                    win[jr][q] = window<j - R + 4 * h>(L, C, Rr);
                });
            }
            static_for<K>([&](auto cc) {
                constexpr int c = decltype(cc)::value;
                constexpr int slot = ((U - c) % K + K) % K;
                uint32_t wv[16];
                load_plane_weights(wq + c * K * NH, wv);
#pragma unroll
                for (int vy = 0; vy < VY; ++vy)
#pragma unroll
                    for (int b = 0; b < K; ++b)
#pragma unroll
                        for (int j = 0; j < 4; ++j)
#pragma unroll
                            for (int h = 0; h < NH; ++h)
                                acc[slot][vy][j] = dot4<SG>(win[vy + b][4 * h + j], wv[b * NH + h],
                                                            acc[slot][vy][j]);
                // this plane's products complete before the next plane's
                // weights are loaded (one weight group live in SGPRs)
                pin8(acc[slot]);
            });
        }

        __builtin_amdgcn_s_setprio(0);
        // output plane q = p - (k - 1) is complete in slot (U + 1) mod k
        constexpr int done = (U + 1) % K;
        const int zo = zb + p - (K - 1);
        if (p >= K - 1 && zo < ze && x_ok) {
#pragma unroll
            for (int vy = 0; vy < VY; ++vy) {
                const int y = y0 + wave * VY + vy;
                if (y >= a.ry1) continue;
                // v_cvt_pk_u8_f32 rounds to nearest even and saturates to
                // [0, 255]; no result lies within 1/(4D) of a tie
                uint32_t packed = 0;
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    packed = __builtin_amdgcn_cvt_pk_u8_f32(
                        fmaf((float)acc[done][vy][j], inv_D, bias), j, packed);
                *reinterpret_cast<uint32_t*>(dst + zo * plane + (int64_t)y * a.X + ox) = packed;
            }
        }
#pragma unroll
        for (int vy = 0; vy < VY; ++vy)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[done][vy][j] = 0;
        __syncthreads();
    };

    // whole groups of k steps (no per-step branch around the ring); steps
    // past the slab's last input plane compute values that are never stored
    // (the planner picks slab depths with P a multiple of k)
    for (int p0 = 0; p0 < P; p0 += K)
        static_for<K>([&](auto uc) { step(p0 + decltype(uc)::value, uc); });
}

template <int K, bool SG>
__global__ __launch_bounds__(kNT) __attribute__((amdgpu_waves_per_eu(Geo4<K>::WAVES)))
void filter_dot4_kernel(VolDesc a,
                                                          const uint32_t* __restrict__ wq,
                                                          uint32_t nblocks)
{
    __shared__ __align__(16) uint32_t lds[2 * Geo4<K>::PLANE_BUF];
    const uint32_t lid = xcd_remap(blockIdx.x, nblocks);
    const uint32_t ntiles = (uint32_t)a.tiles_x * (uint32_t)a.tiles_y;
    dot4_tile<K, SG>(a, wq, (int)(lid % ntiles), (int)(lid / ntiles), lds);
}

// Persistent workgroups over a work queue of (volume, tile-slab) items; the
// packed weights of all filters of the class are in the integer pool.
template <int K, bool SG, int VYO>
__global__ __launch_bounds__(kNT) __attribute__((amdgpu_waves_per_eu(Geo4<K>::WAVES)))
void filter_dot4_batched_kernel(BatchArgs b)
{
    __shared__ __align__(16) uint32_t lds[2 * Geo4<K, VYO>::PLANE_BUF];
    __shared__ uint32_t s_item;
    const uint32_t* pool = reinterpret_cast<const uint32_t*>(b.wipool);
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
        dot4_tile<K, SG, VYO>(a, pool + a.woff, (int)(wi.lid % ntiles), (int)(wi.lid / ntiles),
                              lds);
    }
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(&b.counters[1], 1u) == gridDim.x - 1) {
            atomicExch(&b.counters[0], 0u);
            atomicExch(&b.counters[1], 0u);
        }
    }
}

template <int K, bool SG>
hipError_t launch_k(const FilterJob& j, hipStream_t s)
{
    const ClassGeom g = dot4_geom(K);
    // the output region's tiles and z extent (the whole volume unless a range)
    const int RX = j.roi[3] - j.roi[0], RY = j.roi[4] - j.roi[1], RZ = j.roi[5] - j.roi[2];
    const int64_t ntiles = (int64_t)((RX + g.tx - 1) / g.tx) * ((RY + g.ty - 1) / g.ty);
    // tz = 1 mod k: the slab's tz + k - 1 input planes are whole ring turns
    const void* fn = (const void*)&filter_dot4_kernel<K, SG>;
    const int tz = plan_tz(ntiles, RZ, K, 1, 128, resident_wgs(fn), K);
    const VolDesc a = make_desc(j, tz, g);
    const int64_t nb = ntiles * ((RZ + tz - 1) / tz);
    if (nb > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL((filter_dot4_kernel<K, SG>), dim3((unsigned)nb), dim3(kNT), 0, s, a,
                       j.wq, (uint32_t)nb);
    return hipGetLastError();
}

}  // namespace

ClassGeom dot4_geom(int k, int variant)
{
    ClassGeom g;
    g.tx = kTX;
    g.ty = kWaves * (k <= 3 ? 4 : 2) / (variant ? 2 : 1);
    g.tz_min = 4 > 2 * k ? 4 : 2 * k;
    return g;
}

hipError_t launch_filter_dot4(const FilterJob& j, hipStream_t s)
{
    switch (j.k) {
    case 3: return j.q_signed ? launch_k<3, true>(j, s) : launch_k<3, false>(j, s);
    case 5: return j.q_signed ? launch_k<5, true>(j, s) : launch_k<5, false>(j, s);
    case 7: return j.q_signed ? launch_k<7, true>(j, s) : launch_k<7, false>(j, s);
    }
    return hipErrorInvalidValue;
}

template <int K>
const void* batched_sg(bool sg, int variant)
{
    constexpr int ALT = Geo4<K>::VY_DEFAULT / 2;  // tile variant 1: half the rows
    if (variant)
        return sg ? (const void*)&filter_dot4_batched_kernel<K, true, ALT>
                  : (const void*)&filter_dot4_batched_kernel<K, false, ALT>;
    return sg ? (const void*)&filter_dot4_batched_kernel<K, true, 0>
              : (const void*)&filter_dot4_batched_kernel<K, false, 0>;
}

const void* dot4_batched_kernel(int k, bool sg, int variant)
{
    switch (k) {
    case 3: return batched_sg<3>(sg, variant);
    case 5: return batched_sg<5>(sg, variant);
    case 7: return batched_sg<7>(sg, variant);
    }
    return nullptr;
}

}  // namespace vkt
