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
// travel in the kernel arguments (no device allocation).  A workgroup copies
// a run of 64 rows of one brick, its 64 x 4 threads 4 rows at a time, lanes
// along x; workgroups are numbered so that the same run of all bricks of a
// launch lands on one XCD.  Interior source reads are contiguous
// along x, brick writes contiguous; the address mode is applied per
// coordinate.
#include "vkt_internal.h"

#include <algorithm>
#include <utility>
#include <vector>

namespace vkt {
namespace {

constexpr int kNT = 256;
constexpr int kMaxBricks = 128;

struct BrickArgs {
    const void* src;
    int32_t X, Y, Z;
    int32_t B[3];         // interior cells per brick
    int32_t G[3];         // ghost cells per side
    int32_t nbx, nby;     // bricks along x, y
    int32_t first;        // brick index of dst[0]
    int32_t count;        // bricks of this launch
    int32_t mode;
    void* dst[kMaxBricks];
};

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

// Rows of a brick per workgroup: 64, i.e. 16 per thread row lane.
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
    T* __restrict__ dst = static_cast<T*>(a.dst[bl]);
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

// uint8 bricks whose rows are whole dwords (row length, source row length and
// buffers multiples of 4 bytes): each thread writes whole destination dwords.
// A dword inside the source row is formed from the two aligned source dwords
// it straddles and one byte align (v_alignbyte); dwords that reach past an x
// face of the volume take their four cells through the address mode.  The
// row offsets of the workgroup's 64 rows are resolved once, into LDS.
__global__ __launch_bounds__(kNT) void brick_u8_dword_kernel(BrickArgs a)
{
    __shared__ int64_t s_row[kRowsPerWG];
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
    const int64_t r0 = (int64_t)chunk * kRowsPerWG;
    if (r0 >= nrows) return;  // the whole workgroup (before any barrier)
    const int rows = (int)min((int64_t)kRowsPerWG, nrows - r0);
    const int t = threadIdx.x + 64 * threadIdx.y;
    if (t < rows) {
        const int64_t r = r0 + t;
        const int z = (int)(r / dy), y = (int)(r - (int64_t)z * dy);
        const int sy = brick_addr((int64_t)o[1] + y, a.Y, a.mode);
        const int sz = brick_addr((int64_t)o[2] + z, a.Z, a.mode);
        s_row[t] = (sy | sz) >= 0 ? ((int64_t)sz * a.Y + sy) * a.X : -1;
    }
    __syncthreads();
    const uint8_t* __restrict__ src = static_cast<const uint8_t*>(a.src);
    uint32_t* __restrict__ dst = static_cast<uint32_t*>(a.dst[bl]) + r0 * (dx / 4);
    const int nd = dx / 4;
    // Dword j of a row covers source x in [o[0] + 4 j, o[0] + 4 j + 4); it
    // lies inside the source row for j in [jlo, jhi), the same for every row
    // of the brick.
    const int jlo = o[0] >= 0 ? 0 : min(nd, (3 - o[0]) / 4);
    const int last = a.X - 4 - o[0];  // largest 4 j inside the row
    const int jhi = max(jlo, last >= 0 ? min(nd, last / 4 + 1) : 0);
    const int ni = jhi - jlo, nf = nd - ni;
    // Interior dwords, in batches of kBatch per thread: all loads of a batch
    // are issued before its stores.  A dword at byte offset p is the aligned
    // pair (lo, hi) around it shifted by p & 3 bytes (v_alignbyte; shift 0
    // gives lo).  Rows outside the volume under border read as zero.
    constexpr int kBatch = 8;
    const int n = rows * ni;
    for (int i0 = t; i0 < n; i0 += kBatch * kNT) {
        uint32_t lo[kBatch], hi[kBatch], sh[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const int i = i0 + u * kNT;
            lo[u] = hi[u] = sh[u] = 0;
            const int rl = i < n ? i / ni : 0;
            const int64_t so = s_row[rl];
            if (i < n && so >= 0) {
                const int64_t p = so + o[0] + 4 * (jlo + (i - rl * ni));
                const uint32_t* q = reinterpret_cast<const uint32_t*>(src + (p & ~int64_t(3)));
                sh[u] = (uint32_t)(p & 3);
                lo[u] = q[0];
                // the next aligned dword is inside the row when p is not
                // aligned (rows end on a dword boundary)
                if (sh[u]) hi[u] = q[1];
            }
        }
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const int i = i0 + u * kNT;
            if (i < n) {
                const int rl = i / ni;
                dst[(int64_t)rl * nd + jlo + (i - rl * ni)] =
                    __builtin_amdgcn_alignbyte(hi[u], lo[u], sh[u]);
            }
        }
    }
    // Dwords that reach past an x face: four cells through the address mode.
    const int m = rows * nf;
    for (int i = t; i < m; i += kNT) {
        const int rl = i / nf, jf = i - rl * nf;
        const int j = jf < jlo ? jf : jhi + (jf - jlo);
        const int64_t so = s_row[rl];
        const int sx = o[0] + 4 * j;
        uint32_t v = 0;
        if (so >= 0) {
            for (int c = 0; c < 4; ++c) {
                const int cx = brick_addr((int64_t)sx + c, a.X, a.mode);
                if (cx >= 0) v |= (uint32_t)src[so + cx] << (8 * c);
            }
        }
        dst[(int64_t)rl * nd + j] = v;
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

template <typename T>
hipError_t launch_bricks(BrickArgs& a, const std::vector<void*>& dsts, hipStream_t s)
{
    const int64_t rows_max =
        (int64_t)(std::min(a.B[1], a.Y) + 2 * a.G[1]) * (std::min(a.B[2], a.Z) + 2 * a.G[2]);
    const int64_t chunks = (rows_max + kRowsPerWG - 1) / kRowsPerWG;
    if (chunks * kMaxBricks > INT32_MAX) return hipErrorInvalidValue;
    const int n = (int)dsts.size();
    // uint8 with dword rows everywhere: every brick row a whole number of
    // dwords (the interior width and twice the ghost width multiples of 4,
    // or a single brick along x), source rows too, dword-aligned buffers
    bool dword_rows = false;
    if constexpr (sizeof(T) == 1) {
        dword_rows = a.X % 4 == 0 && (2 * a.G[0]) % 4 == 0 &&
                     (a.nbx == 1 || a.B[0] % 4 == 0) &&
                     reinterpret_cast<uintptr_t>(a.src) % 4 == 0;
        for (void* d : dsts) dword_rows = dword_rows && reinterpret_cast<uintptr_t>(d) % 4 == 0;
    }
    for (int f = 0; f < n; f += kMaxBricks) {
        const int cnt = std::min(kMaxBricks, n - f);
        a.first = f;
        a.count = cnt;
        for (int i = 0; i < cnt; ++i) a.dst[i] = dsts[f + i];
        if (dword_rows)
            hipLaunchKernelGGL(brick_u8_dword_kernel, dim3((unsigned)(chunks * cnt)), dim3(64, 4),
                               0, s, a);
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
