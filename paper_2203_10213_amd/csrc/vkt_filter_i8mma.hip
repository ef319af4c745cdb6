// vkt_filter_i8mma.hip -- ApplyFilter for uint8 volumes with 3x3x3 integer
// filters of signed 8-bit weights, on the matrix cores: exact int8 x int8
// products accumulated in int32 (v_mfma_i32_16x16x64_i8).
//
// Operation (paper Sec. 3.2 "Volume Manipulation"; benchmarked as a blur of
// structured volumes in Sec. 4.3): for every output cell
//   T(x,y,z) = sum_{a,b,c} w[a + 3(b + 3c)] * s(A(x+a-1), A(y+b-1), A(z+c-1)),
//   out      = clamp(floor((2T + D) / 2D), 0, 255).
//
// Eligible jobs (decided on the host): uint8 cells, k = 3, integer weights all
// in [-128, 127], sum |w| <= 2048, 1 <= D <= 2^19, rows of a multiple of 4
// cells, 4-byte aligned buffers.
//
// GEMM embedding, per input plane and filter plane c (D_c += W_c S):
//   M (16 rows)    : output x = x0t + m of a 16-wide x-tile;
//   N (16 columns) : output row y = y0w + n of a wave's 16-row band;
//   K (64)         : the 16-cell windows [x0t, x0t + 16) of input rows
//                    y0w + n + b - 1 (b = 0, 1, 2: three 16-byte K chunks)
//                    and, in the fourth chunk, the 6 cells just outside them
//                    (columns x0t - 1 and x0t + 16 of the same three rows);
//   W_c[m][(b, x')] = w[c][b][x' - x0t - m + 1] (zero outside the filter row),
//   S[(b, x')][n]   = s(x', y0w + n + b - 1) - 128.
// The cells enter as signed bytes s - 128 (one XOR per dword when staged);
// the epilogue adds 128 * sum(w) back.  W_c is the same for every tile: it is
// built once on the host (3 x 64 lanes x 16 bytes) and kept in registers.
// With W as the left operand each lane's four accumulators are 4 consecutive
// x outputs of one row, rounded and packed into one dword store.
//
// Mapping to gfx950:
//  * A workgroup of 4 waves owns a 64 x 64 (x, y) output tile and marches
//    through a z-slab; a wave owns 16 rows x four 16-wide x-tiles.
//  * Each input plane is staged in LDS by direct-to-LDS buffer loads (no
//    register round trip), three plane buffers deep: the loads of plane
//    p + 2 are in flight while plane p is computed.  A buffer holds the 66
//    halo rows of the tile's 64 columns plus one halo dword on either side,
//    as raw bytes (rows padded to 80 bytes, so the 16 lanes of a 16-byte
//    read hit distinct banks).  The loads are issued from inline assembly
//    and waited for with an explicit count (the compiler would otherwise
//    wait for every load in flight before each LDS read).  Dwords at an x
//    face of the volume are loaded as the row's edge dword and permuted in
//    place by the lane that loaded them.
//  * Each wave packs, from LDS, one 16-byte entry per (x-tile, output row
//    of its band) with the edge cells of the three input rows, so a lane
//    reads its whole B operand of an x-tile with one 16-byte LDS read; the
//    cells become signed bytes s - 128 there (one XOR per B register).  The
//    entries are written and read by the same wave (LDS operations of a
//    wave complete in order): no extra workgroup barrier.
//  * Input-stationary z ring: an input plane feeds output planes zi - c + 1,
//    c = 0, 1, 2; three accumulator sets per x-tile, the z loop unrolled by
//    3 so that the ring slots are fixed registers; the c = 0 product starts
//    its set from zero.
//  * Epilogue in FP32 as on the dot-product path: T/D + 1/2 is a multiple of
//    1/(2D), so floor(T/D + 1/2) = round-to-nearest(T * (1/D) + 1/(4D))
//    whenever the FMA's error stays below 1/(4D), which the eligibility
//    bounds guarantee; v_cvt_pk_u8_f32 rounds, saturates and packs.
#include "vkt_internal.h"

#include <utility>

namespace vkt {
namespace {

typedef int32_t i32x4 __attribute__((ext_vector_type(4)));

constexpr int kNT = 256, kWaves = 4;
constexpr int kXT = 4;                        // 16-wide x-tiles per wave
constexpr int kTX = 16 * kXT;                 // tile width
constexpr int kTY = 16 * kWaves;              // tile height
constexpr int kHY = kTY + 2;                  // staged rows per plane
constexpr int kRowDw = 18;                    // staged dwords per row (16 + 2 halo)
constexpr int kPitch = 20;                    // dwords per LDS row (18 + 2 padding)
constexpr int kRowsDw = kHY * kPitch;         // staged rows of one plane
constexpr int kLoads = 6;                     // direct-to-LDS loads per wave per plane
constexpr int kMainDw = kWaves * kLoads * 64; // loaded dwords (rows, then unused)
constexpr int kEdgeDw = kXT * kTY * 4;        // edge entries of one plane (16 bytes each)
constexpr int kBufDw = kMainDw + kEdgeDw;     // one plane buffer
constexpr int kBufs = 3;                      // plane buffers
static_assert(kMainDw >= kRowsDw, "the loads cover the staged rows");
static_assert(kNT == kXT * kTY, "one edge entry per thread");
static_assert(kMainDw % 4 == 0 && kBufDw % 4 == 0, "16-byte aligned LDS regions");

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// One dword per lane from the buffer (rsrc, byte offset voff; offsets at or
// past the size read 0) into LDS at byte address m0 + 4 * lane.
__device__ __attribute__((always_inline)) inline void load_to_lds(u32x4 rsrc, uint32_t voff,
                                                                  uint32_t m0)
{
    asm volatile("s_mov_b32 m0, %2\n\tbuffer_load_dword %0, %1, 0 offen lds"
                 :: "v"(voff), "s"(rsrc), "s"(m0) : "memory", "m0");
}

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

__global__ __launch_bounds__(kNT) __attribute__((amdgpu_waves_per_eu(4)))
void filter_i8mma_kernel(VolDesc a, const i32x4* __restrict__ wm, uint32_t nblocks)
{
    __shared__ __align__(16) uint32_t lds[kBufs * kBufDw];
    const uint32_t lid = xcd_remap(blockIdx.x, nblocks);
    const uint32_t ntiles = (uint32_t)a.tiles_x * (uint32_t)a.tiles_y;
    const int tile = (int)(lid % ntiles), slab = (int)(lid / ntiles);

    const uint8_t* __restrict__ src = static_cast<const uint8_t*>(a.src);
    uint8_t* __restrict__ dst = static_cast<uint8_t*>(a.dst);
    const int t = threadIdx.x, lane = t % 64, wave = t / 64;
    const int x0 = a.rx0 + (tile % a.tiles_x) * kTX, y0 = a.ry0 + (tile / a.tiles_x) * kTY;
    const int zb = a.rz0 + slab * a.tz, ze = min(zb + a.tz, a.rz1);
    const int64_t plane = (int64_t)a.X * a.Y;
    const int32_t plane_bytes = (int32_t)plane;  // < 2^31 (host check)

    // ---- W operands of the three filter planes (one 16-byte piece per lane)
    const i32x4 W0 = wm[lane], W1 = wm[64 + lane], W2 = wm[128 + lane];

    // ---- staging plan, the same (x, y) for every plane of the slab.
    // Load j of wave w fills LDS dwords i = 64 (6 w + j) + lane of a plane
    // buffer: row hy = i / 20, dword d = i % 20 of the row: d < 16 are
    // columns x0 + 4d, d = 16 the right halo dword x0 + 64, d = 17 the left
    // halo dword x0 - 4, d = 18, 19 and i past the rows are padding (read
    // 0).  A dword starting at column X (right face) or left of column 0
    // (left face) is, under each address mode, a permutation of the row's
    // last or first dword (X >= 4): clamp broadcasts the edge cell, mirror
    // reverses, wrap takes the other end's dword, border reads zero.
    // Dwords past the right face feed no stored output.
    const int wv_u = __builtin_amdgcn_readfirstlane(wave);  // wave-uniform copy
    uint32_t soff[kLoads];  // byte offset of the dword to load
    uint32_t ssel[kLoads];  // v_perm_b32 selector for face dwords
    uint32_t face = 0;      // bit j: load j's dword is a face dword
#pragma unroll
    for (int j = 0; j < kLoads; ++j) {
        const int i = 64 * (kLoads * wave + j) + lane;
        const int hy = i / kPitch, d = i % kPitch;
        const bool live = i < kRowsDw && d < kRowDw;
        const int col = d < 16 ? x0 + 4 * d : (d == 16 ? x0 + 64 : x0 - 4);
        const int gy = live ? addr_map((int64_t)y0 - 1 + hy, a.Y, a.mode) : -1;
        const uint32_t row = (uint32_t)(gy < 0 ? 0 : gy) * (uint32_t)a.X;
        uint32_t off = row + (uint32_t)col, sel = 0x03020100u;  // identity
        if (gy >= 0 && (col == a.X || col < 0)) {
            const bool right = col == a.X;
            face |= 1u << j;
            switch (a.mode) {
            case vktAddressModeClamp:  // the edge cell four times
                off = right ? row + (uint32_t)a.X - 4u : row;
                sel = right ? 0x03030303u : 0x00000000u;
                break;
            case vktAddressModeMirror:  // the edge dword reversed
                off = right ? row + (uint32_t)a.X - 4u : row;
                sel = 0x00010203u;
                break;
            case vktAddressModeWrap:  // the other end's dword
                off = right ? row : row + (uint32_t)a.X - 4u;
                break;
            default:
                off = kOutside;
                break;
            }
        }
        soff[j] = gy < 0 ? kOutside : off;
        ssel[j] = sel;
    }
    const bool wave_face = __builtin_amdgcn_ballot_w64(face != 0) != 0;
    // Edge entry packed by this lane: x-tile et = lane / 16, output row ey =
    // 16 wave + lane % 16 of the tile; cells x0t - 1 (LDS byte 16 et - 1, for
    // et = 0 the last byte of the left halo dword) and x0t + 16 (byte
    // 16 et + 16) of staged rows ey, ey + 1, ey + 2.
    const int et = lane / 16, ey = 16 * wave + lane % 16;
    const int lbyte = et == 0 ? 4 * 17 + 3 : 16 * et - 1, rbyte = 16 * et + 16;
    const int ebyte = ey * kPitch * 4;              // staged row ey, byte 0
    const int edw = kMainDw + (et * kTY + ey) * 4;  // LDS dword of the entry

    const uint32_t lds_base = (uint32_t)(uintptr_t)lds;  // LDS byte address
    // issue the loads of input plane zi into plane buffer b
    auto gather = [&](int zi, int b) {
        const int gz = addr_map(zi, a.Z, a.mode);  // -1 only for border: a zero plane
        const uint64_t base = reinterpret_cast<uint64_t>(src) +
                              (gz < 0 ? 0 : (uint64_t)gz * (uint64_t)plane_bytes);
        const u32x4 rs = {(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)base),
                          (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(base >> 32)),
                          (uint32_t)__builtin_amdgcn_readfirstlane(gz < 0 ? 0 : plane_bytes),
                          kRsrcWord3};
        const uint32_t m0 = lds_base + 4u * (uint32_t)(b * kBufDw + 64 * kLoads * wv_u);
#pragma unroll
        for (int j = 0; j < kLoads; ++j) load_to_lds(rs, soff[j], m0 + 256u * j);
    };
    // after this wave's loads of buffer b have completed: permute its face dwords
    auto fix_faces = [&](int b) {
        if (!wave_face) return;
        uint32_t* buf = lds + b * kBufDw + 64 * kLoads * wave + lane;
#pragma unroll
        for (int j = 0; j < kLoads; ++j)
            if (face & (1u << j)) buf[64 * j] = __builtin_amdgcn_perm(buf[64 * j], buf[64 * j], ssel[j]);
    };
    // this wave's edge entries of plane buffer b (its staged rows complete)
    auto edges = [&](int b) {
        uint32_t* buf = lds + b * kBufDw;
        const uint8_t* b8 = reinterpret_cast<const uint8_t*>(buf) + ebyte;
        uint32_t e[6];
#pragma unroll
        for (int jr = 0; jr < 3; ++jr) {
            e[2 * jr] = b8[jr * kPitch * 4 + lbyte];
            e[2 * jr + 1] = b8[jr * kPitch * 4 + rbyte];
        }
        *reinterpret_cast<uint2*>(buf + edw) =
            make_uint2(e[0] | (e[1] << 8) | (e[2] << 16) | (e[3] << 24), e[4] | (e[5] << 8));
    };

    // ---- B operand addresses (bytes within a plane buffer) of x-tile xt:
    // lanes of K chunk g < 3 read input row (16 wave + n + g) at column
    // 16 xt, lanes of chunk 3 the edge entry (xt, 16 wave + n)
    const int n = lane % 16, g = lane / 16;
    const uint32_t bbase = g < 3 ? (uint32_t)((16 * wave + n + g) * kPitch) * 4u
                                 : (uint32_t)(kMainDw + (16 * wave + n) * 4) * 4u;
    const uint32_t bstep = g < 3 ? 16u : (uint32_t)kTY * 16u;

    i32x4 acc[3][kXT];
#pragma unroll
    for (int s = 0; s < 3; ++s)
#pragma unroll
        for (int xt = 0; xt < kXT; ++xt) acc[s][xt] = i32x4{0, 0, 0, 0};

    // output (x, y) of accumulator i of x-tile xt: (x0 + 16 xt + 4 g + i,
    // y0 + 16 wave + n), stored through a buffer resource over the output
    // plane: dwords outside the output region get an offset past the plane,
    // and such stores are dropped
    const int oy = y0 + 16 * wave + n;
    const float inv_D = a.inv_D, bias = a.bias;
    uint32_t ooff[kXT];
#pragma unroll
    for (int xt = 0; xt < kXT; ++xt) {
        const int ox = x0 + 16 * xt + 4 * g;  // rx1 is a multiple of 4
        ooff[xt] = (oy < a.ry1 && ox < a.rx1) ? (uint32_t)oy * (uint32_t)a.X + (uint32_t)ox
                                              : kOutside;
    }
    // rounded outputs of one finished plane, stored one step later (before
    // that step's loads are issued, so that a wait for older loads never
    // waits for these stores' successors)
    uint32_t pend[kXT];
    int pend_z = -1;
    auto flush = [&]() {
        if (pend_z < 0) return;
        const __amdgpu_buffer_rsrc_t ro = __builtin_amdgcn_make_buffer_rsrc(
            dst + (int64_t)pend_z * plane, (short)0, plane_bytes, (int)kRsrcWord3);
#pragma unroll
        for (int xt = 0; xt < kXT; ++xt)
            __builtin_amdgcn_raw_buffer_store_b32(pend[xt], ro, (int)ooff[xt], 0, 0);
        pend_z = -1;
    };

    const int zi_beg = zb - 1;
    const int nz = ze - zb;     // output planes of the slab
    const int P = nz + 2;       // input planes of the slab
    // the W operands are in registers before the first plane load is
    // issued, so that no wait for them lands inside the plane loop
    asm volatile("" :: "v"(W0), "v"(W1), "v"(W2));
    gather(zi_beg, 0);
    if (P > 1) gather(zi_beg + 1, 1);

    // input plane p of the slab in buffer p mod 3 at ring position U = p mod 3
    auto step = [&](int p, auto uc) {
        constexpr int U = decltype(uc)::value;
        constexpr int s0 = U, s1 = (U + 2) % 3, s2 = (U + 1) % 3;
        // plane p's loads were issued two steps ago; after them this wave
        // issued one step's stores and, unless the slab ends, plane p + 1's
        // kLoads loads.  Loads complete in order among themselves, so at most
        // kLoads outstanding operations mean plane p's loads are complete.
        if (p + 1 < P) asm volatile("s_waitcnt vmcnt(6)" ::: "memory");
        else asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        static_assert(kLoads == 6, "the wait count above");
        fix_faces(U);
        __syncthreads();  // plane p complete in LDS; buffer (p + 2) mod 3 free
        flush();
        if (p + 2 < P) gather(zi_beg + p + 2, (U + 2) % 3);
        edges(U);
        // keep the entry stores before the B reads in program order; the LDS
        // executes a wave's operations in order, so the reads see them
        asm volatile("" ::: "memory");
        const char* buf = reinterpret_cast<const char*>(lds + U * kBufDw) + bbase;
        i32x4 B[kXT];
#pragma unroll
        for (int xt = 0; xt < kXT; ++xt) {
            B[xt] = *reinterpret_cast<const i32x4*>(buf + xt * bstep);
            B[xt] ^= (int32_t)0x80808080;  // cells as signed bytes s - 128
        }
        const i32x4 zero = {0, 0, 0, 0};
#pragma unroll
        for (int xt = 0; xt < kXT; ++xt) {
            // filter plane 2 completes output plane p - 2 (slot s2), plane 1
            // adds to p - 1 (s1), plane 0 starts p (s0)
            acc[s2][xt] = __builtin_amdgcn_mfma_i32_16x16x64_i8(W2, B[xt], acc[s2][xt], 0, 0, 0);
            acc[s1][xt] = __builtin_amdgcn_mfma_i32_16x16x64_i8(W1, B[xt], acc[s1][xt], 0, 0, 0);
            acc[s0][xt] = __builtin_amdgcn_mfma_i32_16x16x64_i8(W0, B[xt], zero, 0, 0, 0);
        }
        const int zo = zb + p - 2;
        if (p >= 2 && zo < ze) {
#pragma unroll
            for (int xt = 0; xt < kXT; ++xt) {
                // v_cvt_pk_u8_f32 rounds to nearest even and saturates to
                // [0, 255]; no result lies within 1/(4D) of a tie
                uint32_t packed = 0;
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    packed = __builtin_amdgcn_cvt_pk_u8_f32(
                        fmaf((float)acc[s2][xt][i], inv_D, bias), i, packed);
                pend[xt] = packed;
            }
            pend_z = zo;
        }
    };

    // whole groups of 3 steps (no per-step branch around the ring: slot and
    // buffer are fixed registers and offsets); steps past the slab's last
    // input plane compute values that are never stored (the planner picks
    // slab depths with P a multiple of 3)
    using U0 = std::integral_constant<int, 0>;
    using U1 = std::integral_constant<int, 1>;
    using U2 = std::integral_constant<int, 2>;
    for (int p0 = 0; p0 < P; p0 += 3) {
        step(p0, U0{});
        step(p0 + 1, U1{});
        step(p0 + 2, U2{});
    }
    flush();
}

}  // namespace

ClassGeom i8mma_geom()
{
    ClassGeom g;
    g.tx = kTX;
    g.ty = kTY;
    g.tz_min = 6;
    return g;
}

hipError_t launch_filter_i8mma(const FilterJob& j, hipStream_t s)
{
    if (j.k != 3 || j.fmt != vktDataFormatUInt8 || !j.wm) return hipErrorInvalidValue;
    const ClassGeom g = i8mma_geom();
    const int RX = j.roi[3] - j.roi[0], RY = j.roi[4] - j.roi[1], RZ = j.roi[5] - j.roi[2];
    if (RX % 4 != 0 || j.roi[0] % 4 != 0 || j.X % 4 != 0) return hipErrorInvalidValue;
    const int64_t ntiles = (int64_t)((RX + g.tx - 1) / g.tx) * ((RY + g.ty - 1) / g.ty);
    // tz = 1 mod 3: the slab's tz + 2 input planes are whole ring turns
    const void* fn = (const void*)&filter_i8mma_kernel;
    const int tz = plan_tz(ntiles, RZ, 3, 1, 128, resident_wgs(fn), 3);
    VolDesc a = make_desc(j, tz, g);
    a.bias = j.m8_bias;
    const int64_t nb = ntiles * ((RZ + tz - 1) / tz);
    if (nb > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(filter_i8mma_kernel, dim3((unsigned)nb), dim3(kNT), 0, s, a,
                       reinterpret_cast<const i32x4*>(j.wm), (uint32_t)nb);
    return hipGetLastError();
}

}  // namespace vkt
