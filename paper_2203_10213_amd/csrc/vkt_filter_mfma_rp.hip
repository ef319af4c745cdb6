// vkt_filter_mfma_rp.hip -- ApplyFilter for filters of size 5 and 7 on the
// matrix cores: an implicit GEMM on 32x32x16 MFMA tiles over pairs of output
// rows, with split 16-bit operands and FP32 accumulation.
//
// Operation (paper Sec. 3.2 "Volume Manipulation"; benchmarked as a Gaussian
// blur, Sec. 4.3):
//   T(x,y,z) = sum_{a,b,c} w[a + k(b + k c)] * s(A(x+a-r), A(y+b-r), A(z+c-r)).
//
// GEMM embedding, per input plane zi (D += A * B on 32x32x16 tiles):
//   N (columns n) : row pairs of one x-strip: output rows y0 + 2n + dy,
//                   dy in {0, 1}, of NX = 2 output columns;
//   K (reduction) : (row offset b' in 0..k, input column ax in 0..7) pairs,
//                   two rows per 16-deep chunk; the B operand is the input
//                   window s(x_s - r + ax, y0 + 2n + b' - r, zi), read
//                   straight from the LDS-staged plane;
//   M (rows)      : (filter plane c, dy, output x-offset xo), with
//                   A[(c, dy, xo)][(b', ax)] = w[c][b' - dy][ax - xo]
//                   (zero outside the filter), kept in registers.
// Pairing output rows lets one 16-deep chunk carry two filter rows for both
// rows of a pair: for k = 7 the 49 taps of a (c, dy, xo) row fill 49 of 64
// reduction slots and 28 of the 32 M rows are used (67 % of the products are
// filter taps), and each MFMA does twice the work of a 16x16x32 one for the
// same 1 KB input operand, which halves the LDS reads per output.
//
// z ring in registers: lane l holds D rows 8 (r / 4) + 4 (l / 32) + r % 4
// in its registers r = 0..15.  M row (c, dy, xo) is placed at register
// r = 2 c + dy of lane half xo, so register r of either half accumulates the
// contribution of input plane zi to output plane zi - c + r_f (r_f = filter
// radius).  After each input plane registers 2k-2, 2k-1 hold a finished
// output plane (c = k - 1), and the ring advances by register renaming:
// r <- r - 2 (registers 0 and 1 restart at zero) -- no lane crosses.
//
// Output: for each strip, the finished registers of the two lane halves are
// exchanged with v_permlane32_swap, after which lane l holds output row
// y0 + 2 (l % 32) + l / 32 at the strip's two columns; a wave's four strips
// give each lane 8 consecutive cells of one row, rounded and stored with one
// vector store (no LDS transposition).
//
// A workgroup is 4 waves x 4 strips x 2 columns = a 32-wide, 64-tall tile;
// a wave's 4 strips are adjacent, so two 16-byte LDS reads per (K chunk,
// operand piece) hold all four strips' 16-byte windows (dword offsets 0..3),
// and the products issue products-outer/strips-inner (four independent
// accumulators between dependent MFMAs).
#include "vkt_mfma_common.h"

#include <type_traits>

namespace vkt {
namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
// Pieces of two adjacent cells, packed as the dword pairs they are staged
// as (cell 0 in the low half): the same splitting as split_voxel, with the
// float32 pieces converted two at a time.
template <int PM, typename T>
__device__ inline void split_pair(T s0, T s1, uint32_t* pk)
{
    if constexpr (PM == kF32x3 || PM == kF32x6) {
        const float x0 = (float)s0, x1 = (float)s1;
        const uint32_t hu = (uint32_t)bf16_bits(x0) | ((uint32_t)bf16_bits(x1) << 16);
        const float r0 = x0 - __uint_as_float(hu << 16), r1 = x1 - __uint_as_float(hu & 0xffff0000u);
        const uint32_t lu = (uint32_t)bf16_bits(r0) | ((uint32_t)bf16_bits(r1) << 16);
        pk[0] = hu;
        pk[1] = lu;
        if constexpr (PM == kF32x6) {
            const float t0 = r0 - __uint_as_float(lu << 16), t1 = r1 - __uint_as_float(lu & 0xffff0000u);
            pk[2] = (uint32_t)bf16_bits(t0) | ((uint32_t)bf16_bits(t1) << 16);
        }
    } else {
        uint16_t p0[3], p1[3];
        split_voxel<PM>(s0, p0);
        split_voxel<PM>(s1, p1);
#pragma unroll
        for (int ps = 0; ps < Pieces<PM>::PS; ++ps) pk[ps] = (uint32_t)p0[ps] | ((uint32_t)p1[ps] << 16);
    }
}

// Output transposition rows: 32 floats + 4 of padding (rows two apart fall
// in different banks)
constexpr int kEpiPitch = 36;

template <typename T, int K, int PM>
struct RpCfg {
    using Tin = T;
    using PC = Pieces<PM>;
    static constexpr int R = (K - 1) / 2;
    static_assert(K == 5 || K == 7, "filters of 5 or 7");
    static constexpr int NX = 2;                    // output columns per strip
    static constexpr int WS = 4;                    // strips per wave
    static constexpr int NCH = (K + 2) / 2;         // 16-deep chunks: rows b' = 0..k
    static constexpr int TX = 4 * WS * NX;          // 32 columns per workgroup
    static constexpr int TY = 64;                   // 32 row pairs
    static constexpr int HY = TY + K - 1;           // staged rows
    static constexpr int PITCH = 40;                // staged columns (x0 - r ...)
    static_assert(TX + K - 1 <= PITCH && 8 * 3 + 16 <= PITCH, "staged columns");
    static_assert(2 * 31 + 2 * (NCH - 1) + 1 < HY, "staged rows");
    static constexpr int PLANE = HY * PITCH;
    static constexpr int RFIN = 2 * K - 2;          // finished registers RFIN, RFIN + 1
    // planes whose cells are in flight in registers: two (loads issued two
    // planes ahead) except for 6-product float32, which is short of registers
    static constexpr int PF = PM == kF32x6 ? 1 : 2;
};

// Four consecutive cells at byte offset off (4-byte aligned): one 4-, 8- or
// 16-byte buffer load.
template <typename T>
__device__ inline void buf_load4(__amdgpu_buffer_rsrc_t r, uint32_t off, T (&v)[4])
{
    if constexpr (sizeof(T) == 1) {
        const uint32_t d = (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0);
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = (T)(d >> (8 * j));
    } else if constexpr (sizeof(T) == 2) {
        typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
        const u32x2 d = __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0);
        v[0] = (T)d[0];
        v[1] = (T)(d[0] >> 16);
        v[2] = (T)d[1];
        v[3] = (T)(d[1] >> 16);
    } else {
        const u32x4 d = __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, 0);
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = __uint_as_float(d[j]);
    }
}

template <bool F16>
__device__ inline f32x16 mfma32(u16x8 a, u32x4 b, f32x16 c)
{
    if constexpr (F16)
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a),
                                                      __builtin_bit_cast(f16x8, b), c, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a),
                                                       __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

template <class C>
__device__ void rp_tile(const VolDesc& a, const float* __restrict__ w, int tile, int slab,
                        uint16_t* lds_base, float (*epi)[64][kEpiPitch])
{
    using T = typename C::Tin;
    using PC = typename C::PC;
    constexpr int K = 2 * C::R + 1;
    constexpr int R = C::R;
    constexpr int PM = std::is_same<T, uint8_t>::value ? kU8
                       : std::is_same<T, uint16_t>::value ? kU16
                       : (PC::NPROD == 6 ? kF32x6 : kF32x3);
    constexpr int PLANE = C::PLANE;
    // lds[buffer][piece][row * PITCH + column]
    auto lds = reinterpret_cast<uint16_t(*)[PC::PS][PLANE]>(lds_base);

    const int t = threadIdx.x, lane = t % 64, wave = t / 64;
    const int x0 = a.rx0 + (tile % a.tiles_x) * C::TX, y0 = a.ry0 + (tile / a.tiles_x) * C::TY;
    const int zb = a.rz0 + slab * a.tz, ze = min(zb + a.tz, a.rz1);
    const int64_t plane = (int64_t)a.X * a.Y;
    const int32_t plane_bytes = (int32_t)(plane * (int64_t)sizeof(T));  // < 2^31 (host check)

    // ---- A operand (weights): lane l holds M row l % 32 = (c, dy, xo) and
    // the 8 reduction slots (b' = 2q + l / 32, ax = 0..7) of chunk q
    u16x8 W[C::NCH][PC::NBI];
    {
        const int rho = lane % 32, kg = lane / 32;
        const int r = 4 * (rho / 8) + rho % 4, xo = (rho / 4) % 2;
        const int c = r / 2, dy = r % 2;
#pragma unroll
        for (int q = 0; q < C::NCH; ++q) {
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int b = 2 * q + kg - dy, aa = e - xo;
                float wv = 0.f;
                if (c < K && b >= 0 && b < K && aa >= 0 && aa < K) wv = w[(c * K + b) * K + aa];
                uint16_t p[3];
                split_weight<PM>(wv, a.wscale, p);
#pragma unroll
                for (int bi = 0; bi < PC::NBI; ++bi) W[q][bi][e] = p[bi];
            }
        }
        // pin the pieces in registers: without this the compiler keeps the
        // float weights and splits them again for every plane
#pragma unroll
        for (int q = 0; q < C::NCH; ++q)
#pragma unroll
            for (int bi = 0; bi < PC::NBI; ++bi) {
                u32x4 v = __builtin_bit_cast(u32x4, W[q][bi]);
                asm volatile("" : "+v"(v));
                W[q][bi] = __builtin_bit_cast(u16x8, v);
            }
    }

    // ---- staging of the input plane: PITCH x HY cells from (x0 - r, y0 - r),
    // four adjacent cells (a quad) per thread and step: one 4-cell load when
    // the quad lies inside its source row, else four cell loads through the
    // address mode (quads at the volume's x faces)
    constexpr int NQ = C::PLANE / 4;
    constexpr int NE4 = (NQ + kNT - 1) / kNT;
    static_assert(C::PITCH % 4 == 0, "quads inside rows");
    uint32_t goff[NE4][4];
    uint32_t edge = 0;  // bit i: quad i takes four cell loads
#pragma unroll
    for (int i = 0; i < NE4; ++i) {
        const int e = min(t + i * kNT, NQ - 1);  // repeats the last quad (same values)
        const int hy = (4 * e) / C::PITCH, hx = 4 * e - hy * C::PITCH;
        const int gy = addr_map((int64_t)y0 - R + hy, a.Y, a.mode);
        const int xs = x0 - R + hx;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int gx = addr_map((int64_t)xs + j, a.X, a.mode);
            // cells past the volume edge that only feed zero weights still
            // read a finite value: clamp/wrap/mirror fetch them, border reads 0
            goff[i][j] = (gx < 0 || gy < 0)
                             ? kOutside
                             : ((uint32_t)gy * (uint32_t)a.X + (uint32_t)gx) * (uint32_t)sizeof(T);
        }
        // (a row outside the volume under border mode reads 0 as a quad)
        if (gy >= 0 && (xs < 0 || xs + 3 >= a.X)) edge |= 1u << i;
    }
    // cells of the planes in flight: slot p % PF holds plane p
    T raw[C::PF][NE4][4];
    auto gather = [&](auto slot, int zi) {
        constexpr int S = decltype(slot)::value;
        const int gz = addr_map(zi, a.Z, a.mode);
        const char* base = reinterpret_cast<const char*>(a.src) +
                           (gz < 0 ? 0 : (int64_t)gz * plane_bytes);
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<char*>(base), (short)0, gz < 0 ? 0 : plane_bytes, (int)kRsrcWord3);
#pragma unroll
        for (int i = 0; i < NE4; ++i) {
            if (edge & (1u << i)) {
#pragma unroll
                for (int j = 0; j < 4; ++j) raw[S][i][j] = buf_load<T>(rs, goff[i][j]);
            } else {
                buf_load4<T>(rs, goff[i][0], raw[S][i]);
            }
        }
    };
    auto put = [&](auto slot, auto buf) {
        constexpr int S = decltype(slot)::value, BUF = decltype(buf)::value;
#pragma unroll
        for (int i = 0; i < NE4; ++i) {
            const int e = min(t + i * kNT, NQ - 1);
            uint32_t p01[3], p23[3];
            split_pair<PM>(raw[S][i][0], raw[S][i][1], p01);
            split_pair<PM>(raw[S][i][2], raw[S][i][3], p23);
            typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
#pragma unroll
            for (int ps = 0; ps < PC::PS; ++ps)
                *reinterpret_cast<u32x2*>(&lds[BUF][ps][4 * e]) = u32x2{p01[ps], p23[ps]};
        }
    };

    // ---- output: after the exchange lane l holds row 2 (l % 32) + l / 32 of
    // the tile at the wave's 8 columns; the workgroup's 64 x 32 block goes
    // through LDS (epi[P], double buffered) so that each row is stored by 4
    // consecutive lanes, 8 cells each (whole 128-byte rows per 4 lanes)
    const int erow = 2 * (lane % 32) + lane / 32;
    const int srow = t / 4, scol = 8 * (t % 4);
    const int ys = y0 + srow, xs8 = x0 + scol;
    // rows past the region's last row fall beyond the plane: dropped
    const uint32_t ooff =
        ys < a.ry1 ? ((uint32_t)ys * (uint32_t)a.X + (uint32_t)xs8) * (uint32_t)sizeof(T) : kOutside;
    const bool vec_row = a.vec_ok && xs8 + 8 <= a.rx1;

    f32x16 acc[C::WS];
#pragma unroll
    for (int s = 0; s < C::WS; ++s)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[s][r] = 0.f;

    // lane's B-operand row and first column inside the staged plane
    const int brow = 2 * (lane % 32) + lane / 32;
    const int bcol = 8 * wave;

    const int zi_beg = zb - R, zi_end = ze + R;
    using S0 = std::integral_constant<int, 0>;
    using S1 = std::integral_constant<int, 1>;
    gather(S0{}, zi_beg);
    if constexpr (C::PF == 2) gather(S1{}, min(zi_beg + 1, zi_end - 1));
    put(S0{}, S0{});
    __syncthreads();

    // One input plane zi; P = (zi - zi_beg) % 2 is its LDS buffer and its
    // register slot.  The loads of plane zi + 2 go out first (into the slot
    // plane zi has left), plane zi + 1 (loaded one plane earlier) is staged
    // after the products.
    auto step = [&](auto par, int zi) {
        constexpr int P = decltype(par)::value;
        // register slots of the plane loaded now and of the plane staged
        // after the products
        constexpr int LOAD = C::PF == 2 ? P : 0, STAGE = C::PF == 2 ? P ^ 1 : 0;
        gather(std::integral_constant<int, LOAD>{}, min(zi + C::PF, zi_end - 1));

        // Row segments: lane (n, g) = (l % 32, l / 32) needs, in chunk q, the
        // 16 cells from the wave's first column of staged row 2n + g + 2q,
        // i.e. the row lane (n + 1, g) held in chunk q - 1.  Chunk 0 is read
        // from LDS; chunk q + 1 is chunk q moved down one lane inside each
        // 16-lane row (DPP row_shl:1), the last lane of each row reading its
        // own row from LDS.  seg[ps][h]: dwords 4h .. 4h+3 of the segment.
        auto read_seg = [&](int q, u32x4 (&sg)[PC::PS][2]) {
            const int off = (brow + 2 * q) * C::PITCH + bcol;
#pragma unroll
            for (int ps = 0; ps < PC::PS; ++ps)
#pragma unroll
                for (int h = 0; h < 2; ++h)
                    sg[ps][h] = *reinterpret_cast<const u32x4*>(&lds[P][ps][off + 8 * h]);
        };
        u32x4 seg[2][PC::PS][2];
        // the products at raised wave priority: the issue arbiter prefers
        // this wave's matrix instructions over the other wave's staging and
        // epilogue work (1024^3 7^3: 3.18 -> 3.08 ms)
        __builtin_amdgcn_s_setprio(1);
        read_seg(0, seg[0]);
#pragma unroll
        for (int q = 0; q < C::NCH; ++q) {
            u32x4 (&cur)[PC::PS][2] = seg[q & 1];
            u32x4 (&nxt)[PC::PS][2] = seg[(q + 1) & 1];
            if (q + 1 < C::NCH) {
                if ((lane & 15) == 15) read_seg(q + 1, nxt);
            }
            // strips outer, products inner (dependent 32x32x16 MFMAs issue
            // back to back at full rate with two waves per SIMD), so only one
            // strip window is live: dwords s .. s+3 of the segment
#pragma unroll
            for (int st = 0; st < C::WS; ++st) {
                u32x4 B[PC::PS];
#pragma unroll
                for (int ps = 0; ps < PC::PS; ++ps)
#pragma unroll
                    for (int d = 0; d < 4; ++d) B[ps][d] = cur[ps][(st + d) / 4][(st + d) % 4];
#pragma unroll
                for (int pr = 0; pr < PC::NPROD; ++pr)
                    acc[st] = mfma32<PC::F16>(W[q][PC::prod[pr][1]], B[PC::prod[pr][0]], acc[st]);
            }
            // next chunk's segment (after this chunk's products, so the
            // patch reads have landed)
            if (q + 1 < C::NCH) {
#pragma unroll
                for (int ps = 0; ps < PC::PS; ++ps)
#pragma unroll
                    for (int h = 0; h < 2; ++h)
#pragma unroll
                        for (int d = 0; d < 4; ++d)
                            nxt[ps][h][d] = (uint32_t)__builtin_amdgcn_update_dpp(
                                (int)nxt[ps][h][d], (int)cur[ps][h][d], 0x101, 0xf, 0xf, false);
            }
        }
        // the next plane's cells are split and staged after the products
        __builtin_amdgcn_s_setprio(0);
        __builtin_amdgcn_sched_barrier(0);
        put(std::integral_constant<int, STAGE>{}, std::integral_constant<int, P ^ 1>{});

        // ---- registers RFIN, RFIN + 1 hold output plane zi - r
        const int zo = zi - R;
        const bool out = zo >= zb;
        if (out) {
            float v[8];
#pragma unroll
            for (int st = 0; st < C::WS; ++st) {
                // (element values taken by value: a bit cast of a vector
                // element reference reads element 0 with this compiler)
                const float f0 = acc[st][C::RFIN], f1 = acc[st][C::RFIN + 1];
                const auto pq = __builtin_amdgcn_permlane32_swap(__float_as_uint(f0),
                                                                 __float_as_uint(f1), false, false);
                v[2 * st] = __uint_as_float((uint32_t)pq[0]);      // column 2 st
                v[2 * st + 1] = __uint_as_float((uint32_t)pq[1]);  // column 2 st + 1
            }
            float* e = &epi[P][erow][8 * wave];
            *reinterpret_cast<f32x4*>(e) = f32x4{v[0], v[1], v[2], v[3]};
            *reinterpret_cast<f32x4*>(e + 4) = f32x4{v[4], v[5], v[6], v[7]};
        }
        // ---- advance the ring: filter plane c -> c + 1 is register r -> r + 2
#pragma unroll
        for (int st = 0; st < C::WS; ++st) {
#pragma unroll
            for (int r = 2 * K - 1; r >= 2; --r) acc[st][r] = acc[st][r - 2];
            acc[st][0] = 0.f;
            acc[st][1] = 0.f;
        }
        // the next plane (staged above) and this plane's outputs are complete
        __syncthreads();
        if (out) {
            const float* e = &epi[P][srow][scol];
            const f32x4 lo = *reinterpret_cast<const f32x4*>(e);
            const f32x4 hi = *reinterpret_cast<const f32x4*>(e + 4);
            const float v[8] = {lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
            const __amdgpu_buffer_rsrc_t rd = __builtin_amdgcn_make_buffer_rsrc(
                static_cast<char*>(a.dst) + (int64_t)zo * plane_bytes, (short)0, plane_bytes,
                (int)kRsrcWord3);
            store_row<T, 8>(rd, ooff, v, vec_row, a.rx1 - xs8, a.unscale);
        }
    };
    for (int zi = zi_beg; zi < zi_end; zi += 2) {
        step(S0{}, zi);
        if (zi + 1 < zi_end) step(S1{}, zi + 1);
    }
}

template <class C>
constexpr int rp_lds_elems()
{
    return 2 * C::PC::PS * C::PLANE;
}

template <class C>
__global__ __launch_bounds__(kNT) __attribute__((amdgpu_waves_per_eu(2)))
void filter_mfma_rp_kernel(VolDesc a, const float* __restrict__ w, uint32_t nblocks)
{
    __shared__ __align__(16) uint16_t lds[rp_lds_elems<C>()];
    __shared__ __align__(16) float epi[2][64][kEpiPitch];
    const uint32_t lid = xcd_remap(blockIdx.x, nblocks);
    const uint32_t ntiles = (uint32_t)a.tiles_x * (uint32_t)a.tiles_y;
    rp_tile<C>(a, w, (int)(lid % ntiles), (int)(lid / ntiles), lds, epi);
}

// Persistent workgroups over a queue of (volume, tile-slab) items; the last
// workgroup to finish resets the queue counters.
template <class C>
__global__ __launch_bounds__(kNT) __attribute__((amdgpu_waves_per_eu(2)))
void filter_mfma_rp_batched_kernel(BatchArgs b)
{
    __shared__ __align__(16) uint16_t lds[rp_lds_elems<C>()];
    __shared__ __align__(16) float epi[2][64][kEpiPitch];
    __shared__ uint32_t s_item;
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
        rp_tile<C>(a, b.wpool + a.woff, (int)(wi.lid % ntiles), (int)(wi.lid / ntiles), lds, epi);
        // the next item's staging reuses the LDS buffers
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(&b.counters[1], 1u) == gridDim.x - 1) {
            atomicExch(&b.counters[0], 0u);
            atomicExch(&b.counters[1], 0u);
        }
    }
}

template <class C>
ClassGeom rp_geom()
{
    ClassGeom g;
    g.tx = C::TX;
    g.ty = C::TY;
    g.tz_min = 4 * (2 * C::R + 1);
    return g;
}

template <class C>
hipError_t rp_launch(const FilterJob& j, hipStream_t s)
{
    ClassGeom g;
    g.tx = C::TX;
    g.ty = C::TY;
    g.tz_min = 1;
    const int RX = j.roi[3] - j.roi[0], RY = j.roi[4] - j.roi[1], RZ = j.roi[5] - j.roi[2];
    const int64_t ntiles = (int64_t)((RX + g.tx - 1) / g.tx) * ((RY + g.ty - 1) / g.ty);
    const void* fn = (const void*)&filter_mfma_rp_kernel<C>;
    // (slabs as deep as one round of resident workgroups allows: 1024^3 7^3
    // 3.24 ms with slabs capped at 128 planes, 3.09 ms uncapped)
    const int tz = plan_tz(ntiles, RZ, j.k, 1, 1 << 20, resident_wgs(fn), 1);
    const VolDesc a = make_desc(j, tz, g);
    const int64_t nb = ntiles * ((RZ + tz - 1) / tz);
    if (nb > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL((filter_mfma_rp_kernel<C>), dim3((unsigned)nb), dim3(kNT), 0, s, a, j.wf,
                       (uint32_t)nb);
    return hipGetLastError();
}

template <typename T, int PM>
hipError_t rp_dispatch(const FilterJob& j, hipStream_t s)
{
    switch (j.k) {
    case 5: return rp_launch<RpCfg<T, 5, PM>>(j, s);
    case 7: return rp_launch<RpCfg<T, 7, PM>>(j, s);
    }
    return hipErrorInvalidValue;
}

template <typename T, int PM>
const void* rp_batched(int k)
{
    switch (k) {
    case 5: return (const void*)&filter_mfma_rp_batched_kernel<RpCfg<T, 5, PM>>;
    case 7: return (const void*)&filter_mfma_rp_batched_kernel<RpCfg<T, 7, PM>>;
    }
    return nullptr;
}

template <typename T, int PM>
ClassGeom rp_geom_k(int k)
{
    switch (k) {
    case 5: return rp_geom<RpCfg<T, 5, PM>>();
    case 7: return rp_geom<RpCfg<T, 7, PM>>();
    }
    return ClassGeom{};
}

}  // namespace

const void* mfma_batched_kernel_rp(vktDataFormat f, int k, bool six_products)
{
    switch (f) {
    case vktDataFormatUInt8: return rp_batched<uint8_t, kU8>(k);
    case vktDataFormatUInt16: return rp_batched<uint16_t, kU16>(k);
    case vktDataFormatFloat32:
        return six_products ? rp_batched<float, kF32x6>(k) : rp_batched<float, kF32x3>(k);
    }
    return nullptr;
}

ClassGeom mfma_geom_rp(vktDataFormat f, int k, bool six_products)
{
    switch (f) {
    case vktDataFormatUInt8: return rp_geom_k<uint8_t, kU8>(k);
    case vktDataFormatUInt16: return rp_geom_k<uint16_t, kU16>(k);
    case vktDataFormatFloat32:
        return six_products ? rp_geom_k<float, kF32x6>(k) : rp_geom_k<float, kF32x3>(k);
    }
    return ClassGeom{};
}

hipError_t launch_filter_mfma_rp(const FilterJob& j, bool six_products, hipStream_t s)
{
    switch (j.fmt) {
    case vktDataFormatUInt8: return rp_dispatch<uint8_t, kU8>(j, s);
    case vktDataFormatUInt16: return rp_dispatch<uint16_t, kU16>(j, s);
    case vktDataFormatFloat32:
        return six_products ? rp_dispatch<float, kF32x6>(j, s) : rp_dispatch<float, kF32x3>(j, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace vkt
