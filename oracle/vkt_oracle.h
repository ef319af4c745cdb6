/*
 * vkt_oracle.h -- plain host-side FP64 reference of the volkit ApplyFilter,
 * Fill and FillRange operations (Zellmann, Aguirre, Schulze, "Volkit: A
 * Performance-Portable Computer Vision Library for 3D Volumetric Data").
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU library
 * against the paper.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load it.  It shares no code, header,
 * table or helper with the GPU library, and the GPU library never links it.
 *
 * What it computes (see vkt_oracle.c for the per-function citations):
 *   ApplyFilter -- paper Sec. 3.2 "Volume Manipulation": a derived algorithm
 *     that can be written with Transform, i.e. an independent computation per
 *     output cell.  Here: a direct FP64 sum over the k*k*k taps of the source
 *     neighbourhood of every cell (correlation orientation), with the address
 *     mode applied to out-of-range neighbour coordinates.
 *   Fill / FillRange -- paper Sec. 3.2 "Volume Manipulation" and Fig. 4: set
 *     every cell, or every cell of an axis-aligned region of interest given in
 *     cell coordinates, to one value mapped through the volume's value range.
 *   Resample, Flip -- paper Sec. 3.2 (core and transform algorithms) and the
 *     structured-volume benchmarks of Sec. 4.
 *   BrickDecompose -- paper Sec. 3.2 (domain decomposition algorithms): a
 *     volume split into bricks, optionally with ghost cells around each.
 *
 * Layout: a volume of dims X*Y*Z is a dense array, x fastest:
 *   index(x, y, z) = x + X*(y + Y*z).
 * A filter of odd size k is k*k*k doubles, a fastest:
 *   w[a + k*(b + k*c)] multiplies src(x+a-r, y+b-r, z+c-r), r = (k-1)/2.
 *
 * All functions return 0 on success and a negative value on a bad argument.
 */
#ifndef VKT_ORACLE_H
#define VKT_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { VKTO_U8 = 0, VKTO_U16 = 1, VKTO_F32 = 2, VKTO_F64 = 3 };
enum { VKTO_CLAMP = 0, VKTO_WRAP = 1, VKTO_MIRROR = 2, VKTO_BORDER = 3 };

/* Address map for a neighbour coordinate i on an axis of n cells.
 * Returns the cell index in [0, n), or -1 for BORDER outside the volume. */
int64_t vkto_address(int64_t i, int64_t n, int mode);

/* T(x,y,z) = sum_{a,b,c} w[a + k(b + k c)] * s(A(x+a-r), A(y+b-r), A(z+c-r))
 * for every x, y and for z in [z0, z1).  T and Aabs (may be NULL; the same sum
 * over |w|*|s|) are laid out x fastest with (z - z0) as the slowest index.
 * nthreads <= 0 uses every online core.  src is typed by fmt. */
int vkto_correlate(const void* src, int fmt, int64_t X, int64_t Y, int64_t Z,
                   int k, const double* w, int mode, int64_t z0, int64_t z1,
                   double* T, double* Aabs, int nthreads);

/* The same sum on the half-open box [x0,x1) x [y0,y1) x [z0,z1) of the
 * volume (the address mode still acts at the volume's faces, not the box's).
 * T and Aabs (may be NULL) hold the box, x fastest. */
int vkto_correlate_box(const void* src, int fmt, int64_t X, int64_t Y,
                       int64_t Z, int k, const double* w, int mode, int64_t x0,
                       int64_t y0, int64_t z0, int64_t x1, int64_t y1,
                       int64_t z1, double* T, double* Aabs, int nthreads);

/* The same sum at npts explicit cells; pts holds (x, y, z) triples. */
int vkto_correlate_points(const void* src, int fmt, int64_t X, int64_t Y,
                          int64_t Z, int k, const double* w, int mode,
                          const int64_t* pts, int64_t npts, double* T,
                          double* Aabs);

/* Stored result of a float-weight filter from q = T:
 *   F32: (float)q, round to nearest even;
 *   U8/U16: clamp(floor(q + 1/2), 0, 2^bits - 1)  (half-up). */
int vkto_store_float_filter(const double* q, int64_t n, int out_fmt, void* out);

/* Stored result of an integer-weight filter with divisor D >= 1 from the exact
 * integer sum T:
 *   U8/U16: clamp(floor((2T + D) / (2D)), 0, 2^bits - 1), exact in int64;
 *   F32: (float)(T / D). */
int vkto_store_int_filter(const double* T, int64_t n, int64_t D, int out_fmt,
                          void* out);

/* Raw stored value for Fill of `value` in a volume whose value range is
 * [lo, hi]:  integer formats clamp(floor((value-lo)/(hi-lo)*max + 1/2), 0, max),
 * F32 stores value unchanged.  Integer formats need hi != lo. */
int vkto_fill_raw(double value, double lo, double hi, int fmt, double* raw);

/* Write raw into every cell of the half-open box [x0,x1)*[y0,y1)*[z0,z1). */
int vkto_fill_range(void* dst, int fmt, int64_t X, int64_t Y, int64_t Z,
                    int64_t x0, int64_t y0, int64_t z0, int64_t x1, int64_t y1,
                    int64_t z1, double raw);

/* Resample (paper Sec. 3.2: a core algorithm that changes the size of a
 * volume; benchmarked in Sec. 4 as a downscale by two on every axis).  out
 * (Xo*Yo*Zo doubles, x fastest) receives, for every destination cell, the
 * trilinear interpolation of src at the cell's centre mapped to source cell
 * coordinates, u = (i + 1/2) * n_src / n_dst - 1/2 per axis, neighbours
 * clamped to the volume (for a factor of exactly two: the mean of the
 * 2 x 2 x 2 source block).  Aabs (may be NULL) receives the same
 * interpolation of |src|. */
int vkto_resample_linear(const void* src, int fmt, int64_t X, int64_t Y, int64_t Z,
                         int64_t Xo, int64_t Yo, int64_t Zo, double* out, double* Aabs);

/* Flip (paper Sec. 3.2, a transform algorithm; benchmarked in Sec. 4 along
 * the axis of the longest extent): dst(x) = src(n - 1 - x) along axis
 * (0 = x, 1 = y, 2 = z), every other coordinate unchanged.  dst and src are
 * typed by fmt and must not overlap. */
int vkto_flip(const void* src, int fmt, int64_t X, int64_t Y, int64_t Z, int axis,
              void* dst);

/* One brick of a brick decomposition with ghost cells (paper Sec. 3.2,
 * domain decomposition algorithms): dst is the box of nx*ny*nz cells whose
 * first cell sits at source coordinate (x0, y0, z0) -- which may be negative
 * or reach past the volume, so that the box holds ghost cells around a brick
 * interior -- each cell read through the address map (BORDER outside: 0).
 * dst is typed by fmt, x fastest, and must not overlap src. */
int vkto_brick(const void* src, int fmt, int64_t X, int64_t Y, int64_t Z, int64_t x0,
               int64_t y0, int64_t z0, int64_t nx, int64_t ny, int64_t nz, int mode,
               void* dst);

#ifdef __cplusplus
}
#endif

#endif /* VKT_ORACLE_H */
