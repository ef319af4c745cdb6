/*
 * vkt.h -- C99 interface of libvkt, an MI355X (gfx950) implementation of the
 * structured-volume ApplyFilter path of volkit (Zellmann, Aguirre, Schulze,
 * "Volkit: A Performance-Portable Computer Vision Library for 3D Volumetric
 * Data").
 *
 * Style follows the paper's C99 API (Sec. 3.3 and Fig. 4): a `vkt` prefix,
 * handle out-parameters, a structured volume made of dims, a cell format, a
 * cell size and a value range.  All calls return a vktError; no C++ exception
 * crosses this interface.
 *
 * Volume layout (device memory): dense, x fastest,
 *     index(x, y, z) = x + dimX * (y + dimY * z),
 * cells of 1 (UInt8), 2 (UInt16) or 4 (Float32) bytes.
 *
 * Execution model (paper Sec. 3.1, thread-local ExecutionPolicy): every call
 * enqueues its work on the calling thread's HIP stream (vktSetStream; default
 * the null stream of the current device) and returns after the enqueue.
 * Argument errors are reported synchronously, before anything is enqueued,
 * and leave every output untouched.  Faults of enqueued work surface as
 * vktDeviceError from vktSynchronize or from a later call.
 */
#ifndef VKT_H
#define VKT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum vktError {
    vktNoError = 0,
    vktInvalidValue = 1,   /* bad handle, pointer, size or combination */
    vktOutOfMemory = 2,    /* device allocation failed */
    vktDeviceError = 3,    /* a HIP call or an enqueued kernel failed */
    vktUnsupported = 4     /* valid request that this library cannot run */
} vktError;

typedef enum vktDataFormat {
    vktDataFormatUInt8 = 0,
    vktDataFormatUInt16 = 1,
    vktDataFormatFloat32 = 2
} vktDataFormat;

/* Boundary rule for filter taps that fall outside the volume. */
typedef enum vktAddressMode {
    vktAddressModeClamp = 0,   /* nearest edge cell */
    vktAddressModeWrap = 1,    /* periodic */
    vktAddressModeMirror = 2,  /* reflect about the cell edge (edge repeated) */
    vktAddressModeBorder = 3   /* zero outside */
} vktAddressMode;

/* Arithmetic used by vktApplyFilter on the calling thread, for filters with
 * float weights and k >= 5 (integer-weight filters and k < 5 always run the
 * exact vector-ALU path).  The split modes run the filter as an implicit GEMM
 * on the matrix cores with 16-bit operand pieces and FP32 accumulation:
 * UInt8/UInt16 cells are split exactly into fp16 pieces and the weights into
 * two fp16 pieces (2 or 4 products); Float32 cells and weights are split
 * into bf16 pieces, keeping 3 products (SplitBF16: dropped terms up to
 * 3 * 2^-16 of |w||s| per tap, faster) or 6 (SplitBF16x6 and Auto: dropped
 * terms below 2^-22 of |w||s|). */
typedef enum vktPrecision {
    vktPrecisionAuto = 0,        /* split for k >= 5; 6 products for Float32 */
    vktPrecisionFP32 = 1,        /* FP32 multiply-add on the vector ALUs */
    vktPrecisionSplitBF16 = 2,   /* matrix cores, 3 bf16 products for Float32 */
    vktPrecisionSplitBF16x6 = 3  /* matrix cores, 6 bf16 products for Float32 */
} vktPrecision;

/* Axis of a volume: x (fastest in memory), y, z. */
typedef enum vktAxis {
    vktAxisX = 0,
    vktAxisY = 1,
    vktAxisZ = 2
} vktAxis;

typedef struct vktStructuredVolume_* vktStructuredVolume;
typedef struct vktFilter_* vktFilter;

/* ---- structured volumes (paper Sec. 3.2 "Volume Types", Fig. 4) -------- */

/* Create a volume that owns a zero-filled device buffer of dimX*dimY*dimZ
 * cells on the current device.  cellX/Y/Z is the cell size (metadata).
 * [lo, hi] is the value range that Fill/FillRange map float values through
 * for integer formats (lo != hi required for UInt8/UInt16).
 * Errors: vktInvalidValue for a NULL out-pointer, a dim <= 0, an unknown
 * format or lo == hi on an integer format; vktOutOfMemory. */
vktError vktStructuredVolumeCreate(vktStructuredVolume* volume, int32_t dimX,
                                   int32_t dimY, int32_t dimZ,
                                   vktDataFormat format, float cellX,
                                   float cellY, float cellZ, float lo, float hi);

/* Wrap caller-owned device memory (e.g. a torch tensor) without copying.
 * The library never frees devPtr; the caller keeps it alive until
 * vktStructuredVolumeDestroy has returned and all enqueued work using it has
 * completed.  devPtr must be aligned to the cell size.
 * Errors: as vktStructuredVolumeCreate, plus a NULL or misaligned devPtr. */
vktError vktStructuredVolumeCreateFromDevicePtr(vktStructuredVolume* volume,
                                                int32_t dimX, int32_t dimY,
                                                int32_t dimZ,
                                                vktDataFormat format,
                                                void* devPtr, float lo,
                                                float hi);

/* Release the handle; frees the buffer only if the volume owns it.  The
 * buffer is freed with hipFree, which waits for outstanding work on it. */
vktError vktStructuredVolumeDestroy(vktStructuredVolume volume);

vktError vktStructuredVolumeGetDevicePtr(vktStructuredVolume volume,
                                         void** devPtr);
vktError vktStructuredVolumeGetDims(vktStructuredVolume volume, int32_t* dimX,
                                    int32_t* dimY, int32_t* dimZ);
vktError vktStructuredVolumeGetDataFormat(vktStructuredVolume volume,
                                          vktDataFormat* format);

/* ---- filters (paper Sec. 3.2 "Volume Manipulation": ApplyFilter applies
 *      user-specified convolution kernels such as edge detection or a
 *      Gaussian blur; Sec. 4.3 benchmarks the Gaussian blur) --------------- */

/* A dense k*k*k filter of float weights, copied at creation (host array of
 * k^3 floats, a fastest: w[a + k*(b + k*c)] multiplies the cell at offset
 * (a-r, b-r, c-r), r = (k-1)/2 -- correlation orientation).
 * Errors: vktInvalidValue for NULL pointers or k not odd in [1, 15];
 * vktOutOfMemory. */
vktError vktFilterCreate(vktFilter* filter, int32_t k, const float* weights);

/* A dense k*k*k filter of integer weights with a divisor (the paper's
 * user-specified kernels written as integers, e.g. a box filter with divisor
 * k^3, Sec. 3.2): the result is sum(w*s) / divisor, rounded half-up and
 * saturated for integer formats (computed exactly).  |w| < 2^23, divisor in [1, 2^29].
 * Errors: vktInvalidValue for NULL pointers, k not odd in [1, 15], a weight
 * out of range or a divisor out of range; vktOutOfMemory. */
vktError vktFilterCreateInt(vktFilter* filter, int32_t k, const int32_t* weights,
                            int32_t divisor);

/* Release a filter created by vktFilterCreate / vktFilterCreateInt and its
 * device copies of the weights (create / destroy pairs of handles as in the
 * paper's C99 example, Fig. 4).  Work already enqueued with the filter must
 * have completed (the device buffers are freed with hipFree).
 * Errors: vktInvalidValue for a handle that is not a live filter. */
vktError vktFilterDestroy(vktFilter filter);

/* ---- Fill / FillRange (paper Sec. 3.2 "Volume Manipulation", Fig. 4) ---- */

/* Set every cell to `value`.  Integer formats store
 * clamp(floor((value - lo) / (hi - lo) * max + 1/2), 0, max); Float32 stores
 * value.  Errors: vktInvalidValue for a bad handle. */
vktError vktFill(vktStructuredVolume volume, float value);

/* Set the cells of the half-open region [first, last) (cell coordinates) to
 * `value`, mapped as in vktFill.  An empty region is a no-op.
 * Errors: vktInvalidValue for a bad handle, first > last on an axis, or a
 * region outside the volume. */
vktError vktFillRange(vktStructuredVolume volume, int32_t firstX,
                      int32_t firstY, int32_t firstZ, int32_t lastX,
                      int32_t lastY, int32_t lastZ, float value);

/* The paper's C99 names (Fig. 4); identical to vktFill / vktFillRange. */
vktError vktFillSV(vktStructuredVolume volume, float value);
vktError vktFillRangeSV(vktStructuredVolume volume, int32_t firstX,
                        int32_t firstY, int32_t firstZ, int32_t lastX,
                        int32_t lastY, int32_t lastZ, float value);

/* ---- ApplyFilter (paper Sec. 3.2 "Volume Manipulation", Sec. 4.3) ------- */

/* dst(x,y,z) = sum_{a,b,c} w[a + k(b + k c)] * src(A(x+a-r), A(y+b-r),
 * A(z+c-r)) for every cell, with A the address mode on each axis, then
 * stored in the volumes' format: Float32 as the FP32 result; UInt8/UInt16
 * rounded half-up (floor(q + 1/2)) and saturated; integer-weight filters on
 * integer formats compute floor((2T + D) / (2D)) exactly.
 * dst and src must have equal dims and format and must not overlap.
 * The arithmetic follows the thread's vktPrecision (see vktPrecision).
 * Integer-weight filters always use exact integer arithmetic.
 * Errors: vktInvalidValue for bad handles, mismatched or overlapping volumes
 * or a mode out of range; vktUnsupported when an integer-weight filter's
 * sum |w| * max(format) would exceed 2^30 or one z-plane exceeds 2^31 bytes. */
vktError vktApplyFilter(vktStructuredVolume dst, vktStructuredVolume src,
                        vktFilter filter, vktAddressMode mode);

/* Range version (paper Sec. 3.2: algorithms come with a Range variant that
 * operates on an axis-aligned region of interest given in cell
 * coordinates).  Writes only the cells of dst inside the half-open ROI
 * [first, last) -- the same bounds convention as vktFillRange -- with the
 * values vktApplyFilter would store there; every other cell of dst keeps its
 * contents.  The source is addressed through the whole volume and the
 * address mode (cells just outside the ROI are read, not replaced by the
 * address mode).  An empty ROI (first == last on some axis) enqueues nothing.
 * Errors: as vktApplyFilter; vktInvalidValue when first > last or last
 * exceeds the dims on some axis, or a coordinate is negative. */
vktError vktApplyFilterRange(vktStructuredVolume dst, vktStructuredVolume src,
                             vktFilter filter, int32_t firstX, int32_t firstY,
                             int32_t firstZ, int32_t lastX, int32_t lastY,
                             int32_t lastZ, vktAddressMode mode);

/* Batched form (paper Sec. 4.3 filters every structured dataset of its
 * benchmark set; Sec. 3.2 domain decomposition yields many bricks to filter):
 * dst[i] = ApplyFilter(src[i], filters[i]) for i < n, each
 * pair exactly as vktApplyFilter would compute it, for volumes of different
 * sizes and filters of different k.  The pairs are grouped into arithmetic
 * classes (format, k, path); each class runs as one persistent launch whose
 * workgroups take tile-slabs of all its volumes from a work queue, longest
 * first; the class launches are the parallel nodes of one hipGraph that is
 * launched on the calling thread's stream.  The plan (descriptors, work lists,
 * weight pools, graph) is cached per batch signature -- volume pointers and
 * dims, filter identities, mode, precision and stream -- so a repeated batch
 * is one graph launch.  Outputs must not overlap any volume of the batch.
 * Two calls with the same signature must not run concurrently (they share
 * the plan's work queue).  Calls from several threads are serialised inside
 * the library (planning, graph instantiation and launch run one call at a
 * time; the enqueued work runs concurrently on the callers' streams).  With vktSetAutotune(1) the first plan of a batch
 * size class times, per class, both tile heights of the class kernel at
 * candidate z-slab depths on the real data (this writes the outputs and
 * waits for the stream) and records the fastest tile and depth;
 * VKT_TUNE_CACHE=<file> keeps that table across processes.
 * Errors: as vktApplyFilter for any pair; vktInvalidValue for n < 0, NULL
 * arrays or overlapping outputs; vktOutOfMemory for the plan buffer. */
vktError vktApplyFilterBatched(int32_t n, const vktStructuredVolume* dst,
                               const vktStructuredVolume* src,
                               const vktFilter* filters, vktAddressMode mode);

/* Allocation-free batched form, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, validation and results as
 * vktApplyFilterBatched -- the same class kernels, slab depths (the tuning
 * table's entry, else the default; this call never tunes) and summation
 * order -- but no plan, graph or device buffer is created: the batch's
 * descriptors, work lists, work-queue counters and weight pools go to a
 * static device array of the library, 8 MiB per GPU, held by each GPU the
 * library runs on until the process ends.  Each call uploads that data
 * (counters cleared) with copies on the calling thread's stream and then
 * launches the class kernels one after another on the same stream; it calls
 * no hipMalloc / hipFree and no allocating library routine.  Every call on a
 * GPU shares that GPU's array: calls that overlap on one GPU (from other
 * threads or on other streams) race and must be serialised by the caller;
 * calls in order on one stream are safe.  The host waits only for the
 * previous call's upload to have been read.
 * Limit: the batch's descriptors (one per volume), work items (one per output
 * tile-slab of every volume) and weight pools must fit the 8 MiB array;
 * otherwise vktUnsupported is returned before anything is enqueued.
 * Errors: as vktApplyFilterBatched, plus vktUnsupported for a batch beyond
 * the limit. */
vktError vktApplyFilterBatchedNoAlloc(int32_t n, const vktStructuredVolume* dst,
                                      const vktStructuredVolume* src,
                                      const vktFilter* filters,
                                      vktAddressMode mode);

/* ---- Resample and Flip (paper Sec. 3.2 core and transform algorithms;
 *      Sec. 4 downscales by two and flips along the longest axis) --------- */

/* Resample src onto dst's grid (any dims, same format): dst cell i on an
 * axis of n source and m destination cells takes the source at the cell
 * centre u = (i + 1/2) n / m - 1/2, trilinear between the neighbouring
 * cells, neighbours clamped to the volume (so u outside [0, n - 1] takes the
 * edge cell).  Stored as the FP32 value (Float32) or rounded half-up and
 * saturated (UInt8/UInt16).  When every src dim is twice the dst dim the
 * result is the mean of each 2x2x2 block, exact for integer formats
 * ((sum + 4) / 8, truncated).  Other sizes interpolate in FP32, the
 * sample positions split exactly (integer arithmetic) into cell and
 * fraction, the fraction rounded once to FP32: Float32 within a few FP32
 * roundings of the largest neighbour, integer formats within 1 of the exact
 * rounding.
 * Errors: vktInvalidValue for bad handles, different formats or overlapping
 * buffers. */
vktError vktResample(vktStructuredVolume dst, vktStructuredVolume src);

/* dst = src mirrored along `axis`: dst(x) = src(n - 1 - x) on that axis.
 * dst == src (the same buffer) flips in place; otherwise the buffers must not
 * overlap.  Bit-exact for every format.
 * Errors: vktInvalidValue for bad handles, an axis out of range, different
 * dims or formats, or partly overlapping buffers. */
vktError vktFlip(vktStructuredVolume dst, vktStructuredVolume src, vktAxis axis);

/* The paper's C99 names; identical to vktResample / vktFlip. */
vktError vktResampleSV(vktStructuredVolume dst, vktStructuredVolume src);
vktError vktFlipSV(vktStructuredVolume dst, vktStructuredVolume src, vktAxis axis);

/* ---- BrickDecompose (paper Sec. 3.2 domain decomposition algorithms) ---- */

/* Bricks of (brickX, brickY, brickZ) interior cells tile the volume: brick
 * (bx, by, bz) starts at cell (bx*brickX, by*brickY, bz*brickZ), and the last
 * brick on an axis keeps the remainder, so there are ceil(dim / brick)
 * bricks per axis.  A brick volume holds its interior plus ghost cells on
 * both sides of each axis (ghostX/Y/Z per side), taken from the source
 * through the address mode (border: 0).  With ghosts of at least the filter
 * radius, ApplyFilter on a brick reproduces the whole-volume ApplyFilter on
 * the brick's interior, whatever mode the brick is filtered with.
 * Errors (all three calls): vktInvalidValue for a bad handle or NULL pointer,
 * a brick size < 1 or a ghost width < 0. */
vktError vktBrickDecomposeGetNumBricks(vktStructuredVolume src, int32_t brickX,
                                       int32_t brickY, int32_t brickZ,
                                       int32_t* numX, int32_t* numY,
                                       int32_t* numZ);
/* Dims of brick (bx, by, bz), ghosts included:
 * min(brick, dim - b*brick) + 2*ghost per axis.  vktInvalidValue also for a
 * brick index outside the grid. */
vktError vktBrickDecomposeGetBrickDims(vktStructuredVolume src, int32_t brickX,
                                       int32_t brickY, int32_t brickZ,
                                       int32_t ghostX, int32_t ghostY,
                                       int32_t ghostZ, int32_t bx, int32_t by,
                                       int32_t bz, int32_t* dimX, int32_t* dimY,
                                       int32_t* dimZ);
/* Write every brick: bricks[bx + numX*(by + numY*bz)] for all n =
 * numX*numY*numZ bricks, each a volume of src's format with exactly the
 * dims above (created by the caller, e.g. with vktStructuredVolumeCreate).
 * One launch per 128 bricks, no device allocation.  Errors: as above, and
 * vktInvalidValue when n differs from the brick count, a brick has the wrong
 * dims or format, a mode is out of range, or brick buffers overlap each
 * other or src. */
vktError vktBrickDecompose(int32_t n, const vktStructuredVolume* bricks,
                           vktStructuredVolume src, int32_t brickX,
                           int32_t brickY, int32_t brickZ, int32_t ghostX,
                           int32_t ghostY, int32_t ghostZ, vktAddressMode mode);
/* The paper's C99 name; identical to vktBrickDecompose. */
vktError vktBrickDecomposeSV(int32_t n, const vktStructuredVolume* bricks,
                             vktStructuredVolume src, int32_t brickX,
                             int32_t brickY, int32_t brickZ, int32_t ghostX,
                             int32_t ghostY, int32_t ghostZ, vktAddressMode mode);

/* ---- per-thread execution state (paper Sec. 3.1 ExecutionPolicy) -------- */

/* stream is a hipStream_t (NULL = the default stream). */
vktError vktSetStream(void* stream);
vktError vktGetStream(void** stream);
vktError vktSetPrecision(vktPrecision precision);
vktError vktGetPrecision(vktPrecision* precision);
/* Enable (1) or disable (0) batched-plan autotuning on this thread (default:
 * the VKT_AUTOTUNE environment variable, "1" enables). */
vktError vktSetAutotune(int enable);

/* Rank-1 fast path (opt-in, per thread; default: the VKT_SEPARABLE
 * environment variable, "1" enables).  A filter whose weights factor as
 * w[c][b][a] = t[c] v[b] u[a] -- exactly for integer filters; for float
 * filters every weight to within 2^-20 of itself (so the three passes stay
 * within about 2^-20 sum|w||s| of the dense sum, plus their own FP32
 * rounding) -- then runs as three one-dimensional
 * passes (3k instead of k^3 multiply-adds per cell, FP32 arithmetic), in
 * vktApplyFilter and vktApplyFilterRange.  Integer filters on integer
 * formats take it only while every partial sum stays an exact integer in
 * FP32, so their results are unchanged; float results may differ from the
 * dense sum by rounding (within the float tolerances).  The batched form
 * always runs the dense arithmetic. */
vktError vktSetSeparable(int enable);
vktError vktGetSeparable(int* enable);
/* Exact int8 matrix-core path (opt-in, per thread; default: the
 * VKT_INT8_MATRIX environment variable, "1" enables).  UInt8 volumes filtered with a
 * 3x3x3 integer filter whose weights all lie in [-128, 127] (sum |w| <= 2048,
 * divisor <= 2^19, rows a multiple of 4 cells, 4-byte aligned buffers, and
 * for a range x bounds that are multiples of 4) run as int8 x int8 products
 * with int32 sums on the matrix cores; otherwise they run as 8-bit dot
 * products on the vector ALUs (measured faster on the 512^3 box filter).  Both compute the exact integer sum, so the stored
 * results are identical.  Single-volume calls only (ApplyFilter and
 * ApplyFilterRange); the batched form uses the dot products. */
vktError vktSetInt8Matrix(int enable);
vktError vktGetInt8Matrix(int* enable);
/* Row-pair threshold (per thread; default 2^24 cells, or the
 * VKT_ROW_PAIR_MIN_CELLS environment variable).  Matrix-core jobs with k = 5,
 * and float32 k = 7 with 3 products, whose output region (the whole volume,
 * or the ROI of a range call) has more than `cells` cells run on the 32x32x16
 * row-pair kernel; smaller ones run on 16x16x32 tiles, which measured faster
 * for batches of volumes up to 256^3.  Both compute the same split products;
 * the summation order differs, so float results may differ by rounding
 * (within the stated tolerances).  A batch chooses per volume exactly as the
 * single call would.  Errors: vktInvalidValue for cells < 0 or a NULL
 * out-pointer. */
vktError vktSetRowPairMinCells(int64_t cells);
vktError vktGetRowPairMinCells(int64_t* cells);

/* *separable = 1 if the filter's weights are rank 1 (as above), else 0. */
vktError vktFilterIsSeparable(vktFilter filter, int* separable);

/* Arithmetic path of an ApplyFilter call. */
typedef enum vktFilterPath {
    vktFilterPathVectorFP32 = 0,   /* FP32 multiply-adds on the vector ALUs (exact
                                      int32 sums for integer filters whose FP32
                                      sums could pass 2^24) */
    vktFilterPathDot8 = 1,         /* 8-bit dot products (uint8 cells, small
                                      integer weights), exact int32 sums */
    vktFilterPathInt8Matrix = 2,   /* int8 x int8 matrix-core products, exact */
    vktFilterPathSplitMatrix = 3,  /* 16-bit operand pieces on the matrix cores,
                                      FP32 accumulation */
    vktFilterPathSeparable = 4     /* rank-1 form: three 1-D passes in FP32 */
} vktFilterPath;

/* The path vktApplyFilter(dst, src, filter, mode) would take on the calling
 * thread now (its precision, separable and int8-matrix settings, and the
 * volumes' sizes and alignment), chosen by the same planning code as the
 * call itself; nothing is enqueued.  *products receives the number of
 * partial products per multiply-add on the split matrix path (uint8 cells 2,
 * uint16 4, Float32 3 or 6) and 1 on every other path.  products may be NULL.
 * Ownership: nothing is retained.  Errors: as vktApplyFilter, plus
 * vktInvalidValue for a NULL path. */
vktError vktGetFilterPath(vktStructuredVolume dst, vktStructuredVolume src,
                          vktFilter filter, vktAddressMode mode,
                          vktFilterPath* path, int32_t* products);

/* Wait for the calling thread's stream (the stream of its execution state,
 * paper Sec. 3.1); reports faults of enqueued work as vktDeviceError. */
vktError vktSynchronize(void);

const char* vktGetErrorString(vktError error);

#ifdef __cplusplus
}
#endif

#endif /* VKT_H */
