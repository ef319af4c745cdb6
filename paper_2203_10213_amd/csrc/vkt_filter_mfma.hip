// vkt_filter_mfma.hip -- ApplyFilter for filters of size k >= 5 on the
// matrix cores: an implicit GEMM with split 16-bit operands and FP32
// accumulation.  This file is compiled twice: with VKT_MFMA_SHAPE=16 for
// k <= 7 (16x16x32 tiles, accumulators in VGPRs) and with VKT_MFMA_SHAPE=32
// for k >= 9 (32x32x16 tiles).
//
// Operation (paper Sec. 3.2 "Volume Manipulation"; benchmarked as a Gaussian
// blur, Sec. 4.3):
//   T(x,y,z) = sum_{a,b,c} w[a + k(b + k c)] * s(A(x+a-r), A(y+b-r), A(z+c-r)).
//
// GEMM embedding, per input plane zi (D += A * B on MFMA tiles):
//   M (rows i)    : consecutive output rows y_i of one x-strip of NX = 2
//                   output columns,
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
// The four x-strips a wave owns are adjacent, so one 32-byte LDS read per
// (row block, K chunk, operand piece) holds all four strips' 16-byte windows
// (at dword offsets 0..3).  The finished column group of all of a wave's
// tiles is an 8 x 32 (16x16 tiles) or 8 x 64 (32x32) block of outputs; it is
// transposed through LDS so that each lane rounds and stores 4 or 8 cells of
// one row with one vector store.
//
// Operand splitting: see vkt_mfma_common.h.
#include "vkt_mfma_common.h"

#ifndef VKT_MFMA_SHAPE
#error "compile with -DVKT_MFMA_SHAPE=16 or 32"
#endif

namespace vkt {
namespace {

// MFMA tile shapes.  AXW = input columns per filter row in the K dimension,
// NACC = accumulator registers per lane.
template <int SHAPE> struct Mf;
template <> struct Mf<16> {
    static constexpr int MT = 16, NT = 16, AXW = 8, NACC = 4;
    using acc_t = f32x4;
};
template <> struct Mf<32> {
    static constexpr int MT = 32, NT = 32, AXW = 16, NACC = 16;
    using acc_t = f32x16;
};

// SYV: row blocks per workgroup (tile height variant of the batched form);
// 0 keeps the measured default below.
template <typename T, int K, int PM, int SYV = 0>
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
    static constexpr int WS = 4;                                    // strips per wave
    static_assert(SX == 4 * WS, "four waves");
    // row blocks per workgroup: 2 for both shapes (16x16 tiles with 4 row
    // blocks needed a third more registers, two waves per SIMD instead of
    // three or four, and measured 5-8 % slower)
    // (32x32 tiles: one row block where that brings the kernel down to two
    // waves per SIMD -- 9^3 with uint8 or 3-product float32 operands, 21 %
    // faster on the 1024^3 9^3 workload, and, with the accumulators in
    // VGPRs, every k >= 9 except 6-product float32 with k >= 13:
    // 2048x2048x1024 11^3 uint16 71.5 -> 53.9 ms, 512^3 k = 11 / 13 / 15
    // uint8 1.78 / 1.70 / 1.92 -> 1.34 / 1.35 / 1.67 ms, 512^3 9^3 uint16
    // 2.30 -> 2.02 ms, 1024^3 9^3 six products 22.7 -> 20.6 ms; 6-product
    // 13^3 and 15^3 would spill 37 and 61 registers there and keep the taller
    // tile at one wave)
    static constexpr bool ONE_BLOCK = SHAPE == 32 && (PM != kF32x6 || K <= 11);
    // segment reads of the next (row block, K chunk) group issued before the
    // current group's products: on 16x16 tiles, for uint16 and for 3-product
    // float32 9^3 (224 registers, no spills; 1024^3 12.45 -> 11.77 ms, 512^3
    // 1.66 -> 1.58 ms, bit-identical).  The other 32x32 kernels read each
    // group's segments just before its products: uint8 9^3 / 11^3 measured 1 %
    // slower pipelined, float32 11^3 the same, and 6-product float32 spills.
    static constexpr bool PIPE = SHAPE == 16 || std::is_same<T, uint16_t>::value ||
                                 (std::is_same<T, float>::value && PM != kF32x6 && K <= 9);
    static constexpr int SY_DEFAULT = SHAPE == 16 ? 2 : (ONE_BLOCK ? 1 : 2);
    static constexpr int SY = SYV ? SYV : SY_DEFAULT;
    static constexpr int TX = SX * NX, TY = SY * M::MT;             // 32 x 32 or 32 x 64 tile
    // a lane's 8-column windows of the wave's WS strips span SEGN columns,
    // read as NRD 16-byte pieces
    static constexpr int SEGN = NX * (WS - 1) + 8;
    static constexpr int NRD = (SEGN + 7) / 8;
    static constexpr int PITCH = SHAPE == 16 ? 40 : 48;             // row pitch (cells)
    static_assert(PITCH % 8 == 0, "16-byte aligned rows");
    static_assert(NX * WS * 3 + (SHAPE == 16 ? 0 : 8) + 8 * NRD <= PITCH, "pitch too small");
    static constexpr int HY = TY + K - 1;                           // staged rows
    static constexpr int NE = (PITCH * HY + kNT - 1) / kNT;         // staged cells / thread
    static constexpr int MTW = WS * SY;                             // M tiles per wave
    // waves per SIMD the single-volume kernel is compiled for: 16x16 tiles
    // with uint8 or 3-product float32 operands fit 128 registers (four
    // waves) without spills; uint16 and 6-product float32 would spill there
    // and keep three; 32x32 tiles take what they need (one or two), except
    // the one-block kernels, held to two waves (196-256 registers; 15^3
    // uint16 and 11^3 six-product float32 spill 14 and 15, and measured
    // faster or no slower)
    static constexpr int WAVES =
        SHAPE == 16 ? (PM == kU8 || PM == kF32x3 ? 4 : 3) : (ONE_BLOCK ? 2 : 1);
    // the persistent batched kernels need more registers: three waves for
    // the 16-bit operand classes, the float32 classes as they come
    static constexpr int BWAVES = SHAPE == 16 && (PM == kU8 || PM == kU16) ? 3 : 1;
};

template <int SHAPE, bool F16>
__device__ inline typename Mf<SHAPE>::acc_t mfma(u32x4 a, u16x8 b, typename Mf<SHAPE>::acc_t c)
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

template <class C>
__device__ void mfma_tile(const VolDesc& a, const float* __restrict__ w, int tile, int slab,
                          uint16_t* lds_base, float* epi)
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
    auto lds = reinterpret_cast<uint16_t(*)[PC::PS][C::HY * C::PITCH]>(lds_base);
    const T* __restrict__ src = static_cast<const T*>(a.src);

    const int t = threadIdx.x, lane = t % 64, wave = t / 64;
    const int x0 = a.rx0 + (tile % a.tiles_x) * C::TX, y0 = a.ry0 + (tile / a.tiles_x) * C::TY;
    const int zb = a.rz0 + slab * a.tz, ze = min(zb + a.tz, a.rz1);
    const int64_t plane = (int64_t)a.X * a.Y;
    const int32_t plane_bytes = (int32_t)(plane * (int64_t)sizeof(T));  // < 2^31 (host check)

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
        // finite value: clamp/wrap/mirror fetch them, border reads zero
        goff[i] = (gx < 0 || gy < 0)
                      ? kOutside
                      : ((uint32_t)gy * (uint32_t)a.X + (uint32_t)gx) * (uint32_t)sizeof(T);
        loff[i] = e;
    }
    // gather only issues the loads; the cells are split into their pieces
    // when they are staged (put), after the plane's products, so the loads
    // stay in flight while the matrix cores work
    T raw[C::NE];
    auto gather = [&](int zi) {
        const int gz = addr_map(zi, a.Z, a.mode);
        const char* base = reinterpret_cast<const char*>(src) +
                           (gz < 0 ? 0 : (int64_t)gz * plane_bytes);
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<char*>(base), (short)0, gz < 0 ? 0 : plane_bytes, (int)kRsrcWord3);
#pragma unroll
        for (int i = 0; i < C::NE; ++i) raw[i] = buf_load<T>(rs, goff[i]);
    };
    auto put = [&](int buf) {
#pragma unroll
        for (int i = 0; i < C::NE; ++i) {
            uint16_t p[3];
            split_voxel<PM>(raw[i], p);
#pragma unroll
            for (int ps = 0; ps < PC::PS; ++ps) lds[buf][ps][loff[i]] = p[ps];
        }
    };

    // ---- output block of the wave: its finished columns form an 8 (x) by
    // BY = SY * MT (32 or 64) (y) block; lanes holding a finished column write
    // it to the wave's LDS block (y fastest), then each lane reads its share of
    // one row (8 cells, or 4 of a 32-row block) and stores it
    constexpr int BX = C::WS * C::NX, BY = C::SY * M::MT;
    static_assert(BX == 8 && (BY == 64 || BY == 32 || BY == 16), "8 x 64, 32 or 16 blocks");
    // lane l stores CPL cells of row l % BY (for 32 rows, two lanes per row)
    constexpr int CPL = BX * BY / 64;
    const int jcol = lane % M::NT, gq = lane / M::NT;
    const int xo = jcol - (K - 1) * C::NX;  // finished column group k-1
    const bool fin = xo >= 0 && xo < C::NX;
    float* const blk = epi + wave * BX * BY;
    const int lrow = lane % BY, lpart = lane / BY;
    const int xw = x0 + BX * wave + CPL * lpart, yl = y0 + lrow;
    // rows past the volume's last row fall beyond the plane: dropped
    const uint32_t ooff =
        yl < a.ry1 ? ((uint32_t)yl * (uint32_t)a.X + (uint32_t)xw) * (uint32_t)sizeof(T) : kOutside;
    const bool vec_row = a.vec_ok && xw + CPL <= a.rx1;

    acc_t acc[C::MTW];
#pragma unroll
    for (int m = 0; m < C::MTW; ++m)
#pragma unroll
        for (int r = 0; r < M::NACC; ++r) acc[m][r] = 0.f;

    // lane's A-operand coordinates inside an M tile
    const int ai = lane % M::MT, ag = lane / M::MT;
    const int acol = C::NX * C::WS * wave + (C::SHAPE == 16 ? 0 : 8 * ag);

    const int zi_beg = zb - R, zi_end = ze + R;
    gather(zi_beg);
    put(0);
    __syncthreads();

    for (int zi = zi_beg; zi < zi_end; ++zi) {
        const int cur = (zi - zi_beg) & 1;
        gather(min(zi + 1, zi_end - 1));

        // (row block, K chunk) groups, software pipelined where C::PIPE: the
        // LDS segments of group g + 1 are read while group g's products issue
        constexpr int NG = C::SY * C::NCH;
        u32x4 seg[2][PC::PS][C::NRD];
        auto load_seg = [&](int g, u32x4 (&sg)[PC::PS][C::NRD]) {
            const int yb = g / C::NCH, q = g % C::NCH;
            int b = C::SHAPE == 16 ? q * 4 + ag : q;
            if (b > K - 1) b = K - 1;  // zero weights there; keep A finite
            const int row = yb * M::MT + ai + b;
            // one segment per piece holds the windows of the wave's strips
#pragma unroll
            for (int ps = 0; ps < PC::PS; ++ps)
#pragma unroll
                for (int h = 0; h < C::NRD; ++h)
                    sg[ps][h] = *reinterpret_cast<const u32x4*>(
                        &lds[cur][ps][row * C::PITCH + acol + 8 * h]);
        };
        constexpr bool PIPE = C::PIPE;
        // the products at raised wave priority (the issue arbiter prefers
        // this wave's matrix work over other waves' staging and epilogues)
        __builtin_amdgcn_s_setprio(1);
        load_seg(0, seg[0]);
#pragma unroll
        for (int g = 0; g < NG; ++g) {
            if constexpr (PIPE) {
                if (g + 1 < NG) load_seg(g + 1, seg[(g + 1) & 1]);
                // keep those reads ahead of this group's products
                __builtin_amdgcn_sched_barrier(0);
            } else {
                if (g > 0) load_seg(g, seg[g & 1]);
            }
            const int yb = g / C::NCH, q = g % C::NCH;
            // strip s's window: dwords s .. s+3 of the segment
            u32x4 A[C::WS][PC::PS];
#pragma unroll
            for (int st = 0; st < C::WS; ++st)
#pragma unroll
                for (int ps = 0; ps < PC::PS; ++ps)
#pragma unroll
                    for (int d = 0; d < 4; ++d)
                        A[st][ps][d] = seg[g & 1][ps][(st + d) / 4][(st + d) % 4];
            // products outer, strips inner: consecutive MFMAs are independent
#pragma unroll
            for (int pr = 0; pr < PC::NPROD; ++pr)
#pragma unroll
                for (int st = 0; st < C::WS; ++st)
                    acc[yb * C::WS + st] = mfma<C::SHAPE, PC::F16>(
                        A[st][PC::prod[pr][0]], B[q][PC::prod[pr][1]], acc[yb * C::WS + st]);
        }
        // the next plane's cells are split and staged after the products
        __builtin_amdgcn_s_setprio(0);
        __builtin_amdgcn_sched_barrier(0);
        put(cur ^ 1);

        // ---- column group k-1 holds output plane zi - r
        const int zo = zi - R;
        if (zo >= zb) {
            if (fin) {
#pragma unroll
                for (int m = 0; m < C::MTW; ++m) {
                    const int yb = m / C::WS, st = m % C::WS;
                    float* col = blk + (st * C::NX + xo) * BY + yb * M::MT + 4 * gq;
#pragma unroll
                    for (int qd = 0; qd < M::NACC / 4; ++qd)
                        *reinterpret_cast<f32x4*>(col + 8 * qd) =
                            f32x4{acc[m][4 * qd], acc[m][4 * qd + 1], acc[m][4 * qd + 2],
                                  acc[m][4 * qd + 3]};
                }
            }
            // the wave's own LDS writes complete before its lanes read them
            asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
            float v[CPL];
#pragma unroll
            for (int xl = 0; xl < CPL; ++xl) v[xl] = blk[(CPL * lpart + xl) * BY + lrow];
            const __amdgpu_buffer_rsrc_t rd = __builtin_amdgcn_make_buffer_rsrc(
                static_cast<char*>(a.dst) + (int64_t)zo * plane_bytes, (short)0, plane_bytes,
                (int)kRsrcWord3);
            store_row<T, CPL>(rd, ooff, v, vec_row, a.rx1 - xw, a.unscale);
            asm volatile("" ::: "memory");
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
constexpr int lds_elems()
{
    return 2 * C::PC::PS * C::HY * C::PITCH;
}
// output transposition blocks: 4 waves x 8 x 64 floats (the 32-row blocks of
// 16x16 tiles use half)
constexpr int kEpiFloats = 4 * 8 * 64;

template <class C>
__global__ __launch_bounds__(kNT) __attribute__((amdgpu_waves_per_eu(C::WAVES)))
void filter_mfma_kernel(VolDesc a,
                                                             const float* __restrict__ w,
                                                             uint32_t nblocks)
{
    __shared__ __align__(16) uint16_t lds[lds_elems<C>()];
    __shared__ __align__(16) float epi[kEpiFloats];
    const uint32_t lid = xcd_remap(blockIdx.x, nblocks);
    const uint32_t ntiles = (uint32_t)a.tiles_x * (uint32_t)a.tiles_y;
    mfma_tile<C>(a, w, (int)(lid % ntiles), (int)(lid / ntiles), lds, epi);
}

// Persistent workgroups over a queue of (volume, tile-slab) items; the last
// workgroup to finish resets the queue counters.
template <class C>
__global__ __launch_bounds__(kNT) __attribute__((amdgpu_waves_per_eu(C::BWAVES)))
void filter_mfma_batched_kernel(BatchArgs b)
{
    __shared__ __align__(16) uint16_t lds[lds_elems<C>()];
    __shared__ __align__(16) float epi[kEpiFloats];
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
        mfma_tile<C>(a, b.wpool + a.woff, (int)(wi.lid % ntiles), (int)(wi.lid / ntiles), lds,
                     epi);
    }
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(&b.counters[1], 1u) == gridDim.x - 1) {
            atomicExch(&b.counters[0], 0u);
            atomicExch(&b.counters[1], 0u);
        }
    }
}

#if VKT_MFMA_SHAPE == 16
#define VKT_MFMA_KS(X) X(5) X(7)
#define VKT_MFMA_FN(name) name##_s16
#else
#define VKT_MFMA_KS(X) X(9) X(11) X(13) X(15)
#define VKT_MFMA_FN(name) name##_s32
#endif

template <class C>
ClassGeom geom_of()
{
    ClassGeom g;
    g.tx = C::TX;
    g.ty = C::TY;
    g.tz_min = 4 * (2 * C::R + 1);
    return g;
}

template <class C>
hipError_t launch_cfg(const FilterJob& j, hipStream_t s)
{
    const ClassGeom g = geom_of<C>();
    // the output region's tiles and z extent (the whole volume unless a range)
    const int RX = j.roi[3] - j.roi[0], RY = j.roi[4] - j.roi[1], RZ = j.roi[5] - j.roi[2];
    const int64_t ntiles = (int64_t)((RX + g.tx - 1) / g.tx) * ((RY + g.ty - 1) / g.ty);
    const void* fn = (const void*)&filter_mfma_kernel<C>;
    // (deeper slabs measured slower for the 16x16 tiles, faster for 32x32)
    const int tz = plan_tz(ntiles, RZ, j.k, 1, C::SHAPE == 16 ? 128 : 512,
                           resident_wgs(fn), 1);
    const VolDesc a = make_desc(j, tz, g);
    const int64_t nb = ntiles * ((RZ + tz - 1) / tz);
    if (nb > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL((filter_mfma_kernel<C>), dim3((unsigned)nb), dim3(kNT), 0, s, a, j.wf,
                       (uint32_t)nb);
    return hipGetLastError();
}

template <typename T, int PM>
hipError_t dispatch_k(const FilterJob& j, hipStream_t s)
{
#define VKT_CASE(KK) \
    case KK: return launch_cfg<Cfg<T, KK, PM>>(j, s);
    switch (j.k) { VKT_MFMA_KS(VKT_CASE) }
#undef VKT_CASE
    return hipErrorInvalidValue;
}

// Tile-height variants of the batched kernels: 0 = the default row blocks,
// 1 = the other choice (16x16 tiles: one row block instead of two; 32x32
// tiles: two instead of one, or one instead of two).
template <typename T, int K, int PM>
constexpr int alt_sy()
{
    return Cfg<T, K, PM>::SY_DEFAULT == 2 ? 1 : 2;
}

template <typename T, int PM>
ClassGeom geom_k(int k, int variant = 0)
{
#define VKT_CASE(KK)                                                       \
    case KK:                                                               \
        return variant ? geom_of<Cfg<T, KK, PM, alt_sy<T, KK, PM>()>>()    \
                       : geom_of<Cfg<T, KK, PM>>();
    switch (k) { VKT_MFMA_KS(VKT_CASE) }
#undef VKT_CASE
    return ClassGeom{};
}

template <typename T, int PM>
const void* batched_k(int k, int variant)
{
#define VKT_CASE(KK)                                                                      \
    case KK:                                                                              \
        return variant                                                                    \
                   ? (const void*)&filter_mfma_batched_kernel<Cfg<T, KK, PM, alt_sy<T, KK, PM>()>> \
                   : (const void*)&filter_mfma_batched_kernel<Cfg<T, KK, PM>>;
    switch (k) { VKT_MFMA_KS(VKT_CASE) }
#undef VKT_CASE
    return nullptr;
}

}  // namespace

ClassGeom VKT_MFMA_FN(mfma_geom)(vktDataFormat f, int k, bool six_products, int variant)
{
    switch (f) {
    case vktDataFormatUInt8: return geom_k<uint8_t, kU8>(k, variant);
    case vktDataFormatUInt16: return geom_k<uint16_t, kU16>(k, variant);
    case vktDataFormatFloat32:
        return six_products ? geom_k<float, kF32x6>(k, variant)
                            : geom_k<float, kF32x3>(k, variant);
    }
    return ClassGeom{};
}

hipError_t VKT_MFMA_FN(launch_filter_mfma)(const FilterJob& j, bool six_products, hipStream_t s)
{
    switch (j.fmt) {
    case vktDataFormatUInt8: return dispatch_k<uint8_t, kU8>(j, s);
    case vktDataFormatUInt16: return dispatch_k<uint16_t, kU16>(j, s);
    case vktDataFormatFloat32:
        return six_products ? dispatch_k<float, kF32x6>(j, s) : dispatch_k<float, kF32x3>(j, s);
    }
    return hipErrorInvalidValue;
}

const void* VKT_MFMA_FN(mfma_batched_kernel)(vktDataFormat f, int k, bool six_products,
                                             int variant)
{
    switch (f) {
    case vktDataFormatUInt8: return batched_k<uint8_t, kU8>(k, variant);
    case vktDataFormatUInt16: return batched_k<uint16_t, kU16>(k, variant);
    case vktDataFormatFloat32:
        return six_products ? batched_k<float, kF32x6>(k, variant)
                            : batched_k<float, kF32x3>(k, variant);
    }
    return nullptr;
}

}  // namespace vkt
