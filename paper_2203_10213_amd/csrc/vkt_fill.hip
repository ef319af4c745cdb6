// vkt_fill.hip -- Fill and FillRange (paper Sec. 3.2 "Volume Manipulation",
// Fig. 4): write one raw cell value to every cell, or to every cell of a
// half-open box [first, last).  Pure HBM writes: 16-byte vector stores for
// the aligned interior of each contiguous run, cell stores for the ragged
// head and tail.
#include "vkt_internal.h"

namespace vkt {
namespace {

constexpr int kFillThreads = 256;

// 16 bytes holding the raw cell value repeated, for a run that starts on a
// cell boundary.
__device__ inline uint4 pattern16(uint32_t raw, int cb)
{
    uint32_t w = cb == 1 ? raw * 0x01010101u : (cb == 2 ? raw * 0x00010001u : raw);
    return make_uint4(w, w, w, w);
}

__device__ inline void store_cell(char* p, int cb, uint32_t raw)
{
    if (cb == 1) *reinterpret_cast<uint8_t*>(p) = (uint8_t)raw;
    else if (cb == 2) *reinterpret_cast<uint16_t*>(p) = (uint16_t)raw;
    else *reinterpret_cast<uint32_t*>(p) = raw;
}

// Split [p, p + nbytes) into an unaligned head, a run of 16-byte words and a
// tail.  head and tail are whole cells because p is cell-aligned.
__device__ inline void split16(const char* p, int64_t nbytes, int64_t& head,
                               int64_t& words)
{
    int64_t mis = (int64_t)(reinterpret_cast<uintptr_t>(p) & 15);
    head = mis ? 16 - mis : 0;
    if (head > nbytes) head = nbytes;
    words = (nbytes - head) >> 4;
}

__global__ __launch_bounds__(kFillThreads) void fill_kernel(char* dst,
                                                            int64_t nbytes,
                                                            int cb,
                                                            uint32_t raw)
{
    int64_t head, words;
    split16(dst, nbytes, head, words);
    const uint4 pat = pattern16(raw, cb);
    uint4* body = reinterpret_cast<uint4*>(dst + head);
    const int64_t stride = (int64_t)gridDim.x * kFillThreads;
    for (int64_t i = (int64_t)blockIdx.x * kFillThreads + threadIdx.x; i < words;
         i += stride)
        body[i] = pat;
    if (blockIdx.x == 0) {
        const int64_t tail0 = head + (words << 4);
        for (int64_t b = (int64_t)threadIdx.x * cb; b < head; b += kFillThreads * cb)
            store_cell(dst + b, cb, raw);
        for (int64_t b = tail0 + (int64_t)threadIdx.x * cb; b < nbytes;
             b += kFillThreads * cb)
            store_cell(dst + b, cb, raw);
    }
}

// One block per (y, z) row of the box (grid-stride over rows); the row's
// bytes [first.x, last.x) are written like fill_kernel's run.
__global__ __launch_bounds__(kFillThreads) void fill_range_kernel(
    char* dst, int cb, int32_t X, int32_t Y, int32_t x0, int32_t y0,
    int32_t z0, int32_t nx, int32_t ny, int64_t nrows, uint32_t raw)
{
    const uint4 pat = pattern16(raw, cb);
    for (int64_t row = blockIdx.x; row < nrows; row += gridDim.x) {
        const int64_t y = y0 + row % ny;
        const int64_t z = z0 + row / ny;
        char* p = dst + ((z * Y + y) * X + x0) * cb;
        const int64_t nbytes = (int64_t)nx * cb;
        int64_t head, words;
        split16(p, nbytes, head, words);
        uint4* body = reinterpret_cast<uint4*>(p + head);
        for (int64_t i = threadIdx.x; i < words; i += kFillThreads) body[i] = pat;
        const int64_t tail0 = head + (words << 4);
        for (int64_t b = (int64_t)threadIdx.x * cb; b < head; b += kFillThreads * cb)
            store_cell(p + b, cb, raw);
        for (int64_t b = tail0 + (int64_t)threadIdx.x * cb; b < nbytes;
             b += kFillThreads * cb)
            store_cell(p + b, cb, raw);
    }
}

}  // namespace

hipError_t launch_fill(void* dst, int cb, int64_t n_cells, uint32_t raw,
                       hipStream_t s)
{
    if (n_cells <= 0) return hipSuccess;
    const int64_t words = (n_cells * cb) / 16 + 1;
    int64_t blocks = (words + kFillThreads - 1) / kFillThreads;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(fill_kernel, dim3((unsigned)blocks), dim3(kFillThreads),
                       0, s, static_cast<char*>(dst), n_cells * cb, cb, raw);
    return hipGetLastError();
}

hipError_t launch_fill_range(void* dst, int cb, int32_t X, int32_t Y,
                             const int32_t first[3], const int32_t last[3],
                             uint32_t raw, hipStream_t s)
{
    const int32_t nx = last[0] - first[0], ny = last[1] - first[1],
                  nz = last[2] - first[2];
    if (nx <= 0 || ny <= 0 || nz <= 0) return hipSuccess;
    const int64_t nrows = (int64_t)ny * nz;
    const int64_t blocks = nrows < 16384 ? nrows : 16384;
    hipLaunchKernelGGL(fill_range_kernel, dim3((unsigned)blocks),
                       dim3(kFillThreads), 0, s, static_cast<char*>(dst), cb, X,
                       Y, first[0], first[1], first[2], nx, ny, nrows, raw);
    return hipGetLastError();
}

}  // namespace vkt
