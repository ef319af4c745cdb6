// vkt_brick.hip -- BrickDecompose with ghost cells (paper Sec. 3.2, domain
// decomposition algorithms: a volume split into subgrids, optionally with
// ghost cells around each).
//
// Bricks of (BX, BY, BZ) interior cells tile the volume, brick (bx, by, bz)
// starting at cell (bx BX, by BY, bz BZ); the last brick on an axis keeps the
// remainder.  Each brick volume holds its interior plus (gx, gy, gz) ghost
// cells on both sides of each axis, read from the source through the address
// mode (border: 0).  With ghosts of the filter radius, the brick interiors of
// a filtered brick set equal the whole-volume ApplyFilter, so bricks feed the
// batched form directly.
//
// One launch covers up to kMaxBricks bricks, whose destination pointers
// travel in the kernel arguments (no device allocation), split into 32 low
// and 16 high address bits so that 512 of them fit the 4 KiB argument block.
// Bricks whose rows are whole dwords (every format when rows, ghosts and
// buffers are 4-byte multiples) take the row kernel: 16-byte groups of
// destination dwords from one 16-byte source load plus one dword, byte
// aligned with v_alignbyte; other bricks take the cell kernel, lanes along x.
// The address mode is applied per coordinate.
#include "vkt_internal.h"

#include <algorithm>
#include <utility>
#include <vector>

namespace vkt {
namespace {

constexpr int kNT = 256;
constexpr int kMaxBricks = 512;

struct BrickArgs {
    const void* src;
    int32_t X, Y, Z;
    int32_t B[3];         // interior cells per brick
    int32_t G[3];         // ghost cells per side
    int32_t nbx, nby;     // bricks along x, y
    int32_t first;        // brick index of destination 0
    int32_t count;        // bricks of this launch
    int32_t mode;
    int32_t rows_per_wg;  // row kernel: brick rows per workgroup
    int32_t chunks;       // row kernel: workgroups per brick
    uint32_t dst_lo[kMaxBricks];  // destination addresses, bits 0..31
    uint16_t dst_hi[kMaxBricks];  // and bits 32..47
};
static_assert(sizeof(BrickArgs) <= 4096, "kernel argument block");

// Destination i of the launch as a global-memory pointer (a pointer made
// from an integer would otherwise be generic and take flat stores).
template <typename T>
__device__ inline __attribute__((address_space(1))) T* brick_dst(const BrickArgs& a, int i)
{
    return (__attribute__((address_space(1))) T*)((uintptr_t)a.dst_hi[i] << 32 | a.dst_lo[i]);
}

// Address mode on one axis; -1: outside under border (reads zero).
__device__ inline int brick_addr(int64_t i, int64_t n, int mode)
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

// Workgroup id -> logical id such that consecutive logical ids run on one
// XCD (the dispatcher deals workgroups to the 8 XCDs round-robin, each XCD
// with its own L2).
__device__ inline uint32_t xcd_group(uint32_t b, uint32_t n)
{
    const uint32_t q = n / 8, rem = n % 8, xcd = b % 8, idx = b / 8;
    return xcd < rem ? xcd * (q + 1) + idx : rem * (q + 1) + (xcd - rem) * q + idx;
}

// Cell kernel: rows of a brick per workgroup: 64, i.e. 16 per thread row lane.
constexpr int kRowsPerWG = 64;
constexpr int kRowsPerThread = kRowsPerWG / 4;

template <typename T>
__global__ __launch_bounds__(kNT) void brick_kernel(BrickArgs a)
{
    // logical id = brick + count * chunk: the bricks of one chunk (row run),
    // which share the source cache lines at their x faces, sit on one XCD
    const uint32_t logical = xcd_group(blockIdx.x, gridDim.x);
    const int bl = (int)(logical % (uint32_t)a.count);
    const int chunk = (int)(logical / (uint32_t)a.count);
    const int b = a.first + bl;
    const int bx = b % a.nbx, by = (b / a.nbx) % a.nby, bz = b / (a.nbx * a.nby);
    const int o[3] = {bx * a.B[0] - a.G[0], by * a.B[1] - a.G[1], bz * a.B[2] - a.G[2]};
    const int dx = min(a.B[0], a.X - bx * a.B[0]) + 2 * a.G[0];
    const int dy = min(a.B[1], a.Y - by * a.B[1]) + 2 * a.G[1];
    const int dz = min(a.B[2], a.Z - bz * a.B[2]) + 2 * a.G[2];
    const int64_t nrows = (int64_t)dy * dz;
    const int64_t r0 = (int64_t)chunk * kRowsPerWG + threadIdx.y;
    if (r0 >= nrows) return;
    const T* __restrict__ src = static_cast<const T*>(a.src);
    __attribute__((address_space(1))) T* __restrict__ dst = brick_dst<T>(a, bl);
    // this thread's rows r0 + 4 i: source row offsets (-1: outside, zeros)
    int64_t soff[kRowsPerThread];
#pragma unroll
    for (int i = 0; i < kRowsPerThread; ++i) {
        const int64_t r = r0 + 4 * i;
        soff[i] = -1;
        if (r < nrows) {
            const int z = (int)(r / dy), y = (int)(r - (int64_t)z * dy);
            const int sy = brick_addr((int64_t)o[1] + y, a.Y, a.mode);
            const int sz = brick_addr((int64_t)o[2] + z, a.Z, a.mode);
            if ((sy | sz) >= 0) soff[i] = ((int64_t)sz * a.Y + sy) * a.X;
        }
    }
    // lanes along x; all of the thread's loads of one pass are issued before
    // its stores
    for (int x = threadIdx.x; x < dx; x += 64) {
        const int sx = brick_addr((int64_t)o[0] + x, a.X, a.mode);
        T v[kRowsPerThread];
#pragma unroll
        for (int i = 0; i < kRowsPerThread; ++i)
            v[i] = (soff[i] >= 0 && sx >= 0) ? src[soff[i] + sx] : T(0);
#pragma unroll
        for (int i = 0; i < kRowsPerThread; ++i) {
            const int64_t r = r0 + 4 * i;
            if (r < nrows) dst[r * dx + x] = v[i];
        }
    }
}

// brick_addr in 32-bit arithmetic, for |i| and 2 n below 2^31 (the row
// kernel's launch condition: every extent plus its ghost width at most 2^30).
__device__ inline int brick_addr32(int i, int n, int mode)
{
    if (i >= 0 && i < n) return i;
    if (mode == vktAddressModeClamp) return i < 0 ? 0 : n - 1;
    if (mode == vktAddressModeWrap) {
        const int m = i % n;
        return m < 0 ? m + n : m;
    }
    if (mode == vktAddressModeMirror) {
        const int p = 2 * n;
        int m = i % p;
        if (m < 0) m += p;
        return m < n ? m : p - 1 - m;
    }
    return -1;
}

// Dwords [jlo, jhi) of a brick row whose source bytes lie inside the source
// row: byte origin ob of the brick row in the source row (negative before
// it), source row of xb bytes, nd dwords per brick row.  Rows with fewer
// than 4 such dwords count as all face (jlo = jhi = 0), so that every
// 16-byte group of a row is whole.
__host__ __device__ inline void inside_dwords(int64_t ob, int64_t xb, int nd, int& jlo, int& jhi)
{
    jlo = ob >= 0 ? 0 : (int)min((int64_t)nd, (3 - ob) / 4);
    const int64_t last = xb - 4 - ob;  // largest 4 j inside the row
    jhi = max(jlo, last >= 0 ? (int)min((int64_t)nd, last / 4 + 1) : 0);
    if (jhi - jlo < 4) jlo = jhi = 0;
}

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4a4 __attribute__((ext_vector_type(4), aligned(4)));

// Row kernel items (16-byte groups or face dwords) per thread and pass: 3
// (512^3 into 64^3 bricks + 2 ghosts: uint8 0.082 ms, float32 0.250 ms;
// with 2 items 0.081 / 0.263 ms, with 4 items 0.082 / 0.258 ms, with 1
// item 0.091 / 0.307 ms).
constexpr int kRowItems = 3;

// Row kernel for cells of E bytes: brick rows of whole dwords, source rows
// and buffers 4-byte aligned.  A workgroup takes rows_per_wg rows of one
// brick (workgroups of a brick consecutive and, through the XCD numbering,
// on one XCD); each row is ng 16-byte groups of inside dwords (the last
// group moved back to end at jhi, so that it rewrites up to 12 bytes of its
// neighbour with the same values) and nf face dwords.  Group: one 16-byte
// load at the aligned source dword under its first byte and, when the row
// is not dword aligned in the source, the dword after it (still inside the
// source row, as the last inside byte lies in it); v_alignbyte shifts each
// output dword out of its aligned pair.  Face dword: its 4 / E cells
// through the address mode, loaded unconditionally (cell 0 of the volume
// for cells outside under border) and masked.  All loads of a thread are
// issued before its stores; no LDS, no barrier.
template <int E>
__global__ __launch_bounds__(kNT) void brick_rows_kernel(BrickArgs a)
{
    constexpr int U = kRowItems;
    const uint32_t logical = xcd_group(blockIdx.x, gridDim.x);
    const int bl = (int)(logical / (uint32_t)a.chunks);
    const int chunk = (int)(logical - (uint32_t)bl * (uint32_t)a.chunks);
    const int b = a.first + bl;
    const int bx = b % a.nbx, byz = b / a.nbx, by = byz % a.nby, bz = byz / a.nby;
    const int o[3] = {bx * a.B[0] - a.G[0], by * a.B[1] - a.G[1], bz * a.B[2] - a.G[2]};
    const int dx = min(a.B[0], a.X - bx * a.B[0]) + 2 * a.G[0];
    const int dy = min(a.B[1], a.Y - by * a.B[1]) + 2 * a.G[1];
    const int dz = min(a.B[2], a.Z - bz * a.B[2]) + 2 * a.G[2];
    const int nrows = dy * dz;  // the host keeps brick dwords below 2^31
    const int r0 = chunk * a.rows_per_wg;
    if (r0 >= nrows) return;
    const int rows = min(a.rows_per_wg, nrows - r0);
    const int nd = (int)((int64_t)dx * E / 4);
    const int64_t ob = (int64_t)o[0] * E;
    const int sh = (int)(ob & 3);
    int jlo, jhi;
    inside_dwords(ob, (int64_t)a.X * E, nd, jlo, jhi);
    const int ni = jhi - jlo, ng = (ni + 3) / 4, nf = nd - ni, per_row = ng + nf;
    const uint8_t* __restrict__ src = static_cast<const uint8_t*>(a.src);
    __attribute__((address_space(1))) uint32_t* __restrict__ dst = brick_dst<uint32_t>(a, bl);
    const int t = threadIdx.x + 64 * threadIdx.y;
    const int n = rows * per_row;
    for (int i0 = t; i0 < n; i0 += U * kNT) {
        u32x4 w[U];
        uint32_t e[U];
        int di[U];
        bool face[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + u * kNT;
            w[u] = u32x4{0u, 0u, 0u, 0u};
            e[u] = 0u;
            di[u] = -1;
            face[u] = false;
            if (i < n) {
                const int rl = i / per_row, k = i - rl * per_row;
                const int r = r0 + rl;
                const int z = r / dy, y = r - z * dy;
                const int sy = brick_addr32(o[1] + y, a.Y, a.mode);
                const int sz = brick_addr32(o[2] + z, a.Z, a.mode);
                // source row start in cells; -1: outside under border
                const int64_t so = (sy | sz) >= 0 ? ((int64_t)sz * a.Y + sy) * a.X : -1;
                if (k < ng) {
                    const int j0 = jlo + min(4 * k, ni - 4);
                    di[u] = r * nd + j0;
                    if (so >= 0) {
                        const uint8_t* q = src + (so * E + ob - sh + 4 * (int64_t)j0);
                        w[u] = *reinterpret_cast<const u32x4a4*>(q);
                        if (sh) e[u] = *reinterpret_cast<const uint32_t*>(q + 16);
                    }
                } else {
                    const int jf = k - ng;
                    const int j = jf < jlo ? jf : jhi + (jf - jlo);
                    di[u] = r * nd + j;
                    face[u] = true;
                    uint32_t v = 0u;
#pragma unroll
                    for (int c = 0; c < 4 / E; ++c) {
                        const int cx = brick_addr32(o[0] + j * (4 / E) + c, a.X, a.mode);
                        const bool ok = so >= 0 && cx >= 0;
                        const int64_t ci = ok ? so + cx : 0;
                        uint32_t cell;
                        if constexpr (E == 1) cell = src[ci];
                        else if constexpr (E == 2) cell = reinterpret_cast<const uint16_t*>(src)[ci];
                        else cell = reinterpret_cast<const uint32_t*>(src)[ci];
                        v |= (ok ? cell : 0u) << (8 * E * c);
                    }
                    w[u].x = v;
                }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (di[u] < 0) continue;
            if (face[u]) {
                dst[di[u]] = w[u].x;
                continue;
            }
            const u32x4 v{__builtin_amdgcn_alignbyte(w[u].y, w[u].x, sh),
                          __builtin_amdgcn_alignbyte(w[u].z, w[u].y, sh),
                          __builtin_amdgcn_alignbyte(w[u].w, w[u].z, sh),
                          __builtin_amdgcn_alignbyte(e[u], w[u].w, sh)};
            *reinterpret_cast<__attribute__((address_space(1))) u32x4a4*>(dst + di[u]) = v;
        }
    }
}

int bricks_along(int32_t dim, int32_t b) { return (dim + b - 1) / b; }

// Dims of brick (bx, by, bz) of src with ghosts.
void brick_dims(const vktStructuredVolume_* src, const int32_t B[3], const int32_t G[3],
                const int32_t bi[3], int32_t d[3])
{
    for (int a = 0; a < 3; ++a) d[a] = std::min(B[a], src->dims[a] - bi[a] * B[a]) + 2 * G[a];
}

bool valid_brick_args(const vktStructuredVolume_* src, const int32_t B[3], const int32_t G[3])
{
    if (!live_volume(src)) return false;
    for (int a = 0; a < 3; ++a) {
        if (B[a] < 1 || G[a] < 0) return false;
        // brick dims stay in int32 range
        if ((int64_t)std::min(B[a], src->dims[a]) + 2 * (int64_t)G[a] > INT32_MAX) return false;
    }
    return true;
}

// Row kernel geometry: the largest per-row item count (16-byte groups plus
// face dwords) over the bricks along x, for cells of E bytes.  Only bricks
// within reach of a face differ from the interior ones, so those and one
// interior brick are visited.
int max_row_items(const BrickArgs& a, int E)
{
    const int reach = a.G[0] / a.B[0] + 2;
    int best = 1;
    for (int bx = 0; bx < a.nbx; ++bx) {
        if (bx > reach + 1 && bx < a.nbx - 2 - reach) bx = a.nbx - 2 - reach;
        const int64_t ob = ((int64_t)bx * a.B[0] - a.G[0]) * E;
        const int dx = std::min(a.B[0], a.X - bx * a.B[0]) + 2 * a.G[0];
        const int nd = (int)((int64_t)dx * E / 4);
        int jlo, jhi;
        inside_dwords(ob, (int64_t)a.X * E, nd, jlo, jhi);
        best = std::max(best, (jhi - jlo + 3) / 4 + nd - (jhi - jlo));
    }
    return best;
}

template <typename T>
hipError_t launch_bricks(BrickArgs& a, const std::vector<void*>& dsts, hipStream_t s)
{
    constexpr int E = sizeof(T);
    const int64_t dx_max = std::min(a.B[0], a.X) + 2 * (int64_t)a.G[0];
    const int64_t rows_max =
        (int64_t)(std::min(a.B[1], a.Y) + 2 * a.G[1]) * (std::min(a.B[2], a.Z) + 2 * a.G[2]);
    const int n = (int)dsts.size();
    // destination addresses travel as 48 bits
    for (void* d : dsts)
        if (reinterpret_cast<uintptr_t>(d) >> 48) return hipErrorInvalidValue;
    // row kernel: every brick row a whole number of dwords (the interior and
    // twice the ghost width in bytes multiples of 4, or a single brick along
    // x), source rows too, dword-aligned buffers, brick dwords below 2^31
    bool rows = (int64_t)a.X * E % 4 == 0 && 2 * (int64_t)a.G[0] * E % 4 == 0 &&
                (a.nbx == 1 || (int64_t)a.B[0] * E % 4 == 0) &&
                reinterpret_cast<uintptr_t>(a.src) % 4 == 0 &&
                dx_max * E / 4 * rows_max < ((int64_t)1 << 31);
    // and 32-bit coordinates: every extent plus its ghost width within 2^30
    const int64_t ext[3] = {a.X, a.Y, a.Z};
    for (int k = 0; k < 3; ++k) rows = rows && ext[k] + a.G[k] <= ((int64_t)1 << 30);
    for (void* d : dsts) rows = rows && reinterpret_cast<uintptr_t>(d) % 4 == 0;
    int64_t chunks;
    if (rows) {
        // one pass per workgroup
        a.rows_per_wg = std::max(1, kRowItems * kNT / max_row_items(a, E));
        chunks = (rows_max + a.rows_per_wg - 1) / a.rows_per_wg;
    } else {
        a.rows_per_wg = kRowsPerWG;
        chunks = (rows_max + kRowsPerWG - 1) / kRowsPerWG;
    }
    if (chunks * kMaxBricks > INT32_MAX) return hipErrorInvalidValue;
    a.chunks = (int32_t)chunks;
    for (int f = 0; f < n; f += kMaxBricks) {
        const int cnt = std::min(kMaxBricks, n - f);
        a.first = f;
        a.count = cnt;
        for (int i = 0; i < cnt; ++i) {
            const uintptr_t d = reinterpret_cast<uintptr_t>(dsts[f + i]);
            a.dst_lo[i] = (uint32_t)d;
            a.dst_hi[i] = (uint16_t)(d >> 32);
        }
        if (rows)
            hipLaunchKernelGGL(brick_rows_kernel<E>, dim3((unsigned)(chunks * cnt)), dim3(64, 4), 0,
                               s, a);
        else
            hipLaunchKernelGGL((brick_kernel<T>), dim3((unsigned)(chunks * cnt)), dim3(64, 4), 0,
                               s, a);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace
}  // namespace vkt

using namespace vkt;

extern "C" {

vktError vktBrickDecomposeGetNumBricks(vktStructuredVolume src, int32_t brickX,
                                       int32_t brickY, int32_t brickZ, int32_t* numX,
                                       int32_t* numY, int32_t* numZ)
{
    const int32_t B[3] = {brickX, brickY, brickZ}, G[3] = {0, 0, 0};
    if (!valid_brick_args(src, B, G) || !numX || !numY || !numZ) return vktInvalidValue;
    *numX = bricks_along(src->dims[0], brickX);
    *numY = bricks_along(src->dims[1], brickY);
    *numZ = bricks_along(src->dims[2], brickZ);
    return vktNoError;
}

vktError vktBrickDecomposeGetBrickDims(vktStructuredVolume src, int32_t brickX,
                                       int32_t brickY, int32_t brickZ, int32_t ghostX,
                                       int32_t ghostY, int32_t ghostZ, int32_t bx, int32_t by,
                                       int32_t bz, int32_t* dimX, int32_t* dimY,
                                       int32_t* dimZ)
{
    const int32_t B[3] = {brickX, brickY, brickZ}, G[3] = {ghostX, ghostY, ghostZ};
    if (!valid_brick_args(src, B, G) || !dimX || !dimY || !dimZ) return vktInvalidValue;
    const int32_t bi[3] = {bx, by, bz};
    for (int a = 0; a < 3; ++a)
        if (bi[a] < 0 || bi[a] >= bricks_along(src->dims[a], B[a])) return vktInvalidValue;
    int32_t d[3];
    brick_dims(src, B, G, bi, d);
    *dimX = d[0];
    *dimY = d[1];
    *dimZ = d[2];
    return vktNoError;
}

vktError vktBrickDecompose(int32_t n, const vktStructuredVolume* bricks, vktStructuredVolume src,
                           int32_t brickX, int32_t brickY, int32_t brickZ, int32_t ghostX,
                           int32_t ghostY, int32_t ghostZ, vktAddressMode mode)
{
    const int32_t B[3] = {brickX, brickY, brickZ}, G[3] = {ghostX, ghostY, ghostZ};
    if (!valid_brick_args(src, B, G) || !bricks) return vktInvalidValue;
    if ((int)mode < vktAddressModeClamp || (int)mode > vktAddressModeBorder) return vktInvalidValue;
    const int32_t nb[3] = {bricks_along(src->dims[0], brickX), bricks_along(src->dims[1], brickY),
                           bricks_along(src->dims[2], brickZ)};
    if ((int64_t)nb[0] * nb[1] * nb[2] != n) return vktInvalidValue;
    const int cb = cell_bytes(src->fmt);
    const uintptr_t s0 = (uintptr_t)src->dev;
    const uintptr_t s1 = s0 + (uintptr_t)cb * src->dims[0] * src->dims[1] * src->dims[2];
    std::vector<void*> dsts(n);
    std::vector<std::pair<uintptr_t, uintptr_t>> ranges(n);
    for (int i = 0; i < n; ++i) {
        const vktStructuredVolume_* v = bricks[i];
        if (!live_volume(v) || v->fmt != src->fmt) return vktInvalidValue;
        const int32_t bi[3] = {i % nb[0], (i / nb[0]) % nb[1], i / (nb[0] * nb[1])};
        int32_t d[3];
        brick_dims(src, B, G, bi, d);
        for (int a = 0; a < 3; ++a)
            if (v->dims[a] != d[a]) return vktInvalidValue;
        const uintptr_t d0 = (uintptr_t)v->dev;
        const uintptr_t d1 = d0 + (uintptr_t)cb * d[0] * d[1] * d[2];
        if (d0 < s1 && s0 < d1) return vktInvalidValue;  // overlaps the source
        dsts[i] = v->dev;
        ranges[i] = {d0, d1};
    }
    std::sort(ranges.begin(), ranges.end());
    for (int i = 1; i < n; ++i)
        if (ranges[i].first < ranges[i - 1].second) return vktInvalidValue;  // bricks overlap
    if (n == 0) return vktNoError;
    BrickArgs a{};
    a.src = src->dev;
    a.X = src->dims[0];
    a.Y = src->dims[1];
    a.Z = src->dims[2];
    for (int k = 0; k < 3; ++k) {
        a.B[k] = B[k];
        a.G[k] = G[k];
    }
    a.nbx = nb[0];
    a.nby = nb[1];
    a.mode = (int)mode;
    hipError_t e = hipErrorInvalidValue;
    switch (src->fmt) {
    case vktDataFormatUInt8: e = launch_bricks<uint8_t>(a, dsts, thread_stream()); break;
    case vktDataFormatUInt16: e = launch_bricks<uint16_t>(a, dsts, thread_stream()); break;
    case vktDataFormatFloat32: e = launch_bricks<float>(a, dsts, thread_stream()); break;
    }
    return from_hip(e);
}

vktError vktBrickDecomposeSV(int32_t n, const vktStructuredVolume* bricks,
                             vktStructuredVolume src, int32_t brickX, int32_t brickY,
                             int32_t brickZ, int32_t ghostX, int32_t ghostY, int32_t ghostZ,
                             vktAddressMode mode)
{
    return vktBrickDecompose(n, bricks, src, brickX, brickY, brickZ, ghostX, ghostY, ghostZ,
                             mode);
}

}  // extern "C"
