// vkt_internal.h -- declarations shared by the libvkt translation units.
//
// Nothing here is part of the public C interface (include/vkt.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/vkt.h"

// Handle types of the C interface.
struct vktStructuredVolume_ {
    int32_t dims[3];
    vktDataFormat fmt;
    float cell[3];
    float lo, hi;
    void* dev;
    bool owned;
    int device;
};

struct vktFilter_ {
    int32_t k;
    bool is_int;
    int32_t divisor;
    int64_t sum_abs_int;        // sum |w| for integer filters
    float wscale;               // power of two: max|w| * wscale in [2^14, 2^15)
    uint64_t serial;            // unique per created filter (plan cache keys)
    float* d_wf;                // device float weights (k^3)
    int32_t* d_wi;              // device int weights (k^3), integer filters
    // 8-bit packed copy for the dot-product path (integer filters, k <= 7,
    // weights in [0, 255] or [-128, 127]): k^2 rows of ceil(k/4) dwords
    uint32_t* d_wq;
    bool q_ok, q_signed;
    int64_t sum_int;            // sum w for integer filters
    // int8 matrix-core operands (k = 3, weights in [-128, 127]): per filter
    // plane c the x-Toeplitz W_c as 64 lanes x 16 signed bytes
    bool m8_ok;
    uint32_t* d_wm;
    // rank-1 factors (u over x | v over y | t over z, 16 floats each) with
    // u (x) v (x) t = w (exactly, with integer factors, for integer filters)
    bool sep_ok;
    int64_t sep_sum_abs;        // sum|u| sum|v| sum|t|
    float* d_sep;
    int device;
};


namespace vkt {

// Number of bytes of one cell of a format.
inline int cell_bytes(vktDataFormat f)
{
    return f == vktDataFormatUInt8 ? 1 : (f == vktDataFormatUInt16 ? 2 : 4);
}

// Divisor-by-multiplication constants for an unsigned 32-bit divisor d >= 1
// (Granlund & Montgomery, "Division by invariant integers using
// multiplication", PLDI 1994, Fig. 4.1): for every 32-bit n,
//   t = umulhi(m, n);  n / d == (t + ((n - t) >> sh1)) >> sh2.
struct UDiv {
    uint32_t m;
    uint32_t sh1;
    uint32_t sh2;
};
UDiv make_udiv(uint32_t d);

// Device weight buffers (per filter, and the batched pools) end with this
// many zero dwords, so that a wide scalar load of the last weight group stays
// inside the allocation.
constexpr int kWeightPad = 16;

// Everything one single-volume ApplyFilter launch needs.
struct FilterJob {
    const void* src;
    void* dst;
    int32_t X, Y, Z;
    int32_t mode;            // vktAddressMode
    vktDataFormat fmt;       // format of src and dst
    int32_t k;
    const float* wf;         // device, k^3 float weights (float path)
    const int32_t* wi;       // device, k^3 int weights (integer path)
    bool int_filter;         // weights are integers with divisor D
    bool int_acc;            // integer accumulation (integer cells, int weights)
    int32_t D;
    UDiv div2D;              // for 2*D
    float inv_D;             // 1/D for float outputs of integer filters
    bool vec_store;          // dst rows can take 16-B-aligned vector stores
    float wscale;            // 2^s with max|w| * 2^s in [2^14, 2^15) (fp16 splitting)
    int32_t roi[6];          // output region [x0, y0, z0, x1, y1, z1)
    bool dot4;               // uint8 cells, 8-bit packed integer weights
    bool q_signed;           // signed 8-bit weights (cells enter as s - 128)
    const uint32_t* wq;      // device packed weights
    float q_bias;            // epilogue constant of the dot-product path
    bool i8mma;              // uint8 cells, k = 3, int8 matrix-core path
    const uint32_t* wm;      // device W operands of that path
    float m8_bias;           // its epilogue constant: (1/4 + 128 sum(w)) / D
    bool sep;                // rank-1 filter on the separable path
    const float* wsep;       // device factors u | v | t (16 floats each)
};

// Stored-result rule of an ApplyFilter.
enum : int32_t {
    kEpiFloat = 0,        // float32 cells, float weights: store T
    kEpiFloatDiv = 1,     // float32 cells, integer weights: store T / D
    kEpiRound = 2,        // integer cells, float weights: floor(T + 1/2), saturate
    kEpiIntDiv = 3        // integer cells, integer weights: floor((2T + D) / 2D)
};

// Per-volume descriptor shared by the single-volume launches (passed by value)
// and the batched persistent kernels (an array in device memory).  Weights are
// addressed as pool + woff so that they stay scalar loads from a kernel
// argument.
struct VolDesc {
    const void* src;
    void* dst;
    int32_t X, Y, Z;
    int32_t mode;
    int32_t tz;              // output planes per z-slab
    int32_t tiles_x, tiles_y;
    uint32_t woff;           // first weight of this volume's filter in the pool
    int32_t epi;             // stored-result rule (kEpi*)
    int32_t D;
    UDiv div2D;
    float inv_D;
    int32_t vec_ok;
    float wscale, unscale;   // fp16 weight scaling of the matrix-core path
    float bias;              // dot-product path: 1/(4D) (+ 128 sum(w) / D)
    int32_t rx0, ry0, rz0;   // output region: tiles start here ...
    int32_t rx1, ry1, rz1;   // ... and outputs stop here (exclusive)
};

// One work item of a batched launch: a tile-slab of one volume.
struct WorkItem {
    uint32_t vol;
    uint32_t lid;            // slab * tiles_x * tiles_y + tile
};

// *p as a wave-uniform value: each dword is read by every lane and taken from
// the first, so the struct (written by the host before the launch) lives in
// scalar registers instead of one copy per lane.
template <typename S>
__device__ inline S uniform_load(const S* p)
{
    static_assert(sizeof(S) % 4 == 0, "whole dwords");
    constexpr int N = sizeof(S) / 4;
    const uint32_t* src = reinterpret_cast<const uint32_t*>(p);
    uint32_t tmp[N];
#pragma unroll
    for (int i = 0; i < N; ++i) tmp[i] = (uint32_t)__builtin_amdgcn_readfirstlane((int)src[i]);
    S out;
    __builtin_memcpy(&out, tmp, sizeof(S));
    return out;
}

// Arguments of a batched persistent kernel (one arithmetic class).
struct BatchArgs {
    const VolDesc* vols;
    const WorkItem* items;   // sorted longest first
    uint32_t nitems;
    uint32_t* counters;      // [0] next item, [1] finished workgroups; both
                             // return to 0 when the launch ends
    const float* wpool;      // float weights of all filters of the class
    const int32_t* wipool;   // int weights (integer accumulation class)
};

// Tile geometry of a kernel class (for planning).
struct ClassGeom {
    int tx, ty;              // output tile in x and y
    int tz_min;              // smallest useful slab depth
};

// Kernel launchers (return the launch status).
hipError_t launch_fill(void* dst, int cell_bytes, int64_t n_cells,
                       uint32_t raw_bits, hipStream_t s);
hipError_t launch_fill_range(void* dst, int cell_bytes, int32_t X, int32_t Y,
                             const int32_t first[3], const int32_t last[3],
                             uint32_t raw_bits, hipStream_t s);
hipError_t launch_filter_valu(const FilterJob& j, hipStream_t s);
// Resample src (dims in) to dst (dims out), same format; Flip along axis
// (0 = x, 1 = y, 2 = z), in place when src == dst.
hipError_t launch_resample(const void* src, void* dst, vktDataFormat f, const int32_t in[3],
                           const int32_t out[3], hipStream_t s);
hipError_t launch_flip(const void* src, void* dst, vktDataFormat f, const int32_t dims[3],
                       int axis, hipStream_t s);
// Rank-1 filters as three one-dimensional passes (opt-in, vktSetSeparable).
hipError_t launch_filter_sep(const FilterJob& j, hipStream_t s);
// 8-bit dot-product path for uint8 volumes with small integer filters.
hipError_t launch_filter_dot4(const FilterJob& j, hipStream_t s);
const void* dot4_batched_kernel(int k, bool q_signed, int variant = 0);
ClassGeom dot4_geom(int k, int variant = 0);
// Exact int8 matrix-core path for uint8 volumes with 3x3x3 filters of signed
// 8-bit weights (single-volume launches).
hipError_t launch_filter_i8mma(const FilterJob& j, hipStream_t s);
ClassGeom i8mma_geom();
// Bytes of the W operand table of that path (3 filter planes x 64 lanes x 16).
constexpr int kI8mmaTableBytes = 3 * 64 * 16;
// Dwords of packed weights per filter on the dot-product path.
inline int dot4_words(int k) { return k * k * ((k + 3) / 4); }
// Matrix-core path for float-weight filters with k >= 5.  six_products
// selects the 6-product bf16 split for float32 volumes (else 3 products).
hipError_t launch_filter_mfma(const FilterJob& j, bool six_products, hipStream_t s);

// The matrix-core kernels are built twice: 16x16x32 tiles for k <= 7 (_s16)
// and 32x32x16 tiles for k >= 9 (_s32); the unsuffixed functions dispatch.
hipError_t launch_filter_mfma_s16(const FilterJob& j, bool six_products, hipStream_t s);
// Single-volume launches with k = 5 or 7: 32x32x16 tiles over pairs of
// output rows (vkt_filter_mfma_rp.hip).
hipError_t launch_filter_mfma_rp(const FilterJob& j, bool six_products, hipStream_t s);
// its persistent batched kernel (one tile shape: both tile-height variants
// are this kernel) and geometry
const void* mfma_batched_kernel_rp(vktDataFormat f, int k, bool six_products);
ClassGeom mfma_geom_rp(vktDataFormat f, int k, bool six_products);
hipError_t launch_filter_mfma_s32(const FilterJob& j, bool six_products, hipStream_t s);
// variant: tile height of the batched kernels (0: the default row blocks,
// 1: the other choice; see kTileVariants)
const void* mfma_batched_kernel_s16(vktDataFormat f, int k, bool six_products, int variant);
const void* mfma_batched_kernel_s32(vktDataFormat f, int k, bool six_products, int variant);
ClassGeom mfma_geom_s16(vktDataFormat f, int k, bool six_products, int variant = 0);
ClassGeom mfma_geom_s32(vktDataFormat f, int k, bool six_products, int variant = 0);

// Batched persistent kernels: the kernel function of a class (for launches
// and graph kernel nodes, taking one BatchArgs by value), its geometry, and
// the workgroup count that fills the device once.
// Tile-height variants of every batched class: 0 = the default tile, 1 = a
// tile half (matrix-core 32x32 tiles: twice) as tall; the autotuner times both.
constexpr int kTileVariants = 2;
const void* valu_batched_kernel(vktDataFormat f, int k, bool int_acc, int variant = 0);
ClassGeom valu_geom(int k, int variant = 0);
// Matrix-core job on the row-pair kernel (k = 5 and 3-product float32
// k = 7, output regions above the thread's row-pair threshold) rather than on
// 16x16x32 tiles; the batched form takes the choice per volume, as its class.
bool mfma_row_pairs(const FilterJob& j, bool six_products);
const void* mfma_batched_kernel(vktDataFormat f, int k, bool six_products, bool row_pairs,
                                int variant = 0);
ClassGeom mfma_geom(vktDataFormat f, int k, bool six_products, bool row_pairs, int variant = 0);
// Fill in the descriptor fields the kernels derive from a FilterJob.
VolDesc make_desc(const FilterJob& j, int tz, ClassGeom g);
// Workgroups of 256 threads of `func` resident on the whole current device
// at once (occupancy x compute units), cached per (kernel, device).
int resident_wgs(const void* func);
// Z-slab depth of a single-volume launch of ntiles tiles per plane: the
// depth in [tz_min, tz_max] (tz = 1 mod `mod` when mod > 1) that minimises
// rounds x (tz + k - 1), where a round is one wave of `slots` resident
// workgroups and tz + k - 1 input planes are streamed per tile-slab.
int plan_tz(int64_t ntiles, int Z, int k, int tz_min, int tz_max, int slots, int mod);

// Validation and planning shared by the single and batched calls: fills j
// and the chosen path (mfma, six products) for one (dst, src, filter) triple.
// roi: output region [x0, y0, z0, x1, y1, z1), NULL for the whole volume
// (validated by the caller); allow_sep: the call has a separable kernel.
vktError build_job(const vktStructuredVolume_* dst, const vktStructuredVolume_* src,
                   const vktFilter_* filt, int mode, vktPrecision prec, FilterJob& j,
                   bool& mfma, bool& six, const int32_t* roi = nullptr,
                   bool allow_sep = true);
bool live_volume(const vktStructuredVolume_* v);
bool live_filter(const vktFilter_* f);
vktError from_hip(hipError_t e);
hipStream_t thread_stream();
vktPrecision thread_precision();
bool thread_autotune();
bool thread_separable();
bool thread_int8_matrix();
int64_t thread_row_pair_min_cells();

}  // namespace vkt
