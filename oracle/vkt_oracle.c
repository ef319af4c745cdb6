/*
 * vkt_oracle.c -- plain, slow, obviously correct FP64 reference for the volkit
 * ApplyFilter / Fill / FillRange operations.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the CPU
 * baseline of the benchmark; never by the GPU library (they share no code).
 *
 * Paper: Zellmann, Aguirre, Schulze, "Volkit: A Performance-Portable Computer
 * Vision Library for 3D Volumetric Data".
 *
 * Readings of the paper used here (the paper states only that ApplyFilter
 * applies user-given convolution kernels such as edge detection or a Gaussian
 * blur, that it can be expressed with Transform -- one callback per cell --
 * and that a faster implementation must not change the behaviour; Sec. 3.2
 * "Volume Manipulation"):
 *   - correlation orientation: tap (a,b,c) reads src(x+a-r, y+b-r, z+c-r);
 *   - odd k, centre tap at r = (k-1)/2;
 *   - the boundary rule is the caller's address mode (clamp, wrap, mirror with
 *     the edge cell repeated, or zero border);
 *   - the filter acts on the raw stored cell values;
 *   - integer results are rounded half-up and saturated to the format range.
 */
#include "vkt_oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

/* ---- cell access ------------------------------------------------------- */

static double load_cell(const void* src, int fmt, int64_t i)
{
    switch (fmt) {
    case VKTO_U8:  return (double)((const uint8_t*)src)[i];
    case VKTO_U16: return (double)((const uint16_t*)src)[i];
    case VKTO_F32: return (double)((const float*)src)[i];
    case VKTO_F64: return ((const double*)src)[i];
    }
    return 0.0;
}

static int valid_fmt(int fmt) { return fmt >= VKTO_U8 && fmt <= VKTO_F64; }

/* ---- address map (boundary rule) ---------------------------------------- */

int64_t vkto_address(int64_t i, int64_t n, int mode)
{
    if (n <= 0) return -1;
    if (i >= 0 && i < n) return i;
    switch (mode) {
    case VKTO_CLAMP:
        return i < 0 ? 0 : n - 1;
    case VKTO_WRAP: {
        int64_t m = i % n;
        return m < 0 ? m + n : m;
    }
    case VKTO_MIRROR: {
        /* ... c b a | a b c ... : reflection about the cell edge, so the edge
         * cell is repeated; the extension has period 2n. */
        int64_t p = 2 * n;
        int64_t m = i % p;
        if (m < 0) m += p;
        return m < n ? m : p - 1 - m;
    }
    case VKTO_BORDER:
    default:
        return -1;
    }
}

/* ---- ApplyFilter: per-cell direct sum ----------------------------------- */

/* One output cell: the Transform-style body (one independent computation per
 * cell, paper Sec. 3.2 "Volume Manipulation"). */
static void one_cell(const void* src, int fmt, int64_t X, int64_t Y, int64_t Z,
                     int k, const double* w, int mode, int64_t x, int64_t y,
                     int64_t z, double* T, double* A)
{
    const int r = (k - 1) / 2;
    double t = 0.0, aabs = 0.0;
    for (int c = 0; c < k; ++c) {
        int64_t zz = vkto_address(z + c - r, Z, mode);
        for (int b = 0; b < k; ++b) {
            int64_t yy = vkto_address(y + b - r, Y, mode);
            for (int a = 0; a < k; ++a) {
                int64_t xx = vkto_address(x + a - r, X, mode);
                double s = 0.0; /* BORDER: cells outside read as zero */
                if (xx >= 0 && yy >= 0 && zz >= 0)
                    s = load_cell(src, fmt, xx + X * (yy + Y * zz));
                double wv = w[a + k * (b + k * c)];
                t += wv * s;
                aabs += fabs(wv) * fabs(s);
            }
        }
    }
    *T = t;
    if (A) *A = aabs;
}

static int check_filter_args(const void* src, int fmt, int64_t X, int64_t Y,
                             int64_t Z, int k, const double* w, int mode)
{
    if (!src || !w || !valid_fmt(fmt)) return -1;
    if (X <= 0 || Y <= 0 || Z <= 0) return -1;
    if (k < 1 || (k % 2) == 0) return -1;
    if (mode < VKTO_CLAMP || mode > VKTO_BORDER) return -1;
    return 0;
}

typedef struct {
    const void* src; int fmt; int64_t X, Y, Z; int k; const double* w; int mode;
    int64_t x0, y0, z0, x1, y1, z1; /* the output box, half-open */
    double* T; double* A;
    int64_t zbeg, zend; /* this worker's planes */
} job_t;

static void* worker(void* p)
{
    job_t* j = (job_t*)p;
    const int64_t nx = j->x1 - j->x0, ny = j->y1 - j->y0;
    for (int64_t z = j->zbeg; z < j->zend; ++z)
        for (int64_t y = j->y0; y < j->y1; ++y)
            for (int64_t x = j->x0; x < j->x1; ++x) {
                int64_t o = ((z - j->z0) * ny + (y - j->y0)) * nx + (x - j->x0);
                one_cell(j->src, j->fmt, j->X, j->Y, j->Z, j->k, j->w, j->mode,
                         x, y, z, &j->T[o], j->A ? &j->A[o] : NULL);
            }
    return NULL;
}

/* Every cell of the half-open box, the z range split over nthreads threads
 * (each cell is independent, so the split changes no result). */
static int correlate_box(const void* src, int fmt, int64_t X, int64_t Y,
                         int64_t Z, int k, const double* w, int mode,
                         int64_t x0, int64_t y0, int64_t z0, int64_t x1,
                         int64_t y1, int64_t z1, double* T, double* Aabs,
                         int nthreads)
{
    if (check_filter_args(src, fmt, X, Y, Z, k, w, mode)) return -1;
    if (!T || x0 < 0 || y0 < 0 || z0 < 0 || x1 > X || y1 > Y || z1 > Z ||
        x0 > x1 || y0 > y1 || z0 > z1)
        return -1;
    if (nthreads <= 0) nthreads = (int)sysconf(_SC_NPROCESSORS_ONLN);
    if (nthreads < 1) nthreads = 1;
    int64_t nz = z1 - z0;
    if (nz == 0 || x0 == x1 || y0 == y1) return 0;
    if (nthreads > nz) nthreads = (int)nz;

    job_t* jobs = (job_t*)calloc((size_t)nthreads, sizeof(job_t));
    pthread_t* th = (pthread_t*)calloc((size_t)nthreads, sizeof(pthread_t));
    if (!jobs || !th) { free(jobs); free(th); return -2; }
    for (int t = 0; t < nthreads; ++t) {
        job_t j = {src, fmt, X, Y, Z, k, w, mode, x0, y0, z0, x1, y1, z1, T, Aabs,
                   z0 + nz * t / nthreads, z0 + nz * (t + 1) / nthreads};
        jobs[t] = j;
    }
    int started = 0;
    for (int t = 1; t < nthreads; ++t)
        if (pthread_create(&th[t], NULL, worker, &jobs[t]) == 0) started = t;
        else break;
    worker(&jobs[0]);
    for (int t = 1; t <= started; ++t) pthread_join(th[t], NULL);
    /* planes of workers that failed to start are computed here */
    for (int t = started + 1; t < nthreads; ++t) worker(&jobs[t]);
    free(jobs);
    free(th);
    return 0;
}

int vkto_correlate(const void* src, int fmt, int64_t X, int64_t Y, int64_t Z,
                   int k, const double* w, int mode, int64_t z0, int64_t z1,
                   double* T, double* Aabs, int nthreads)
{
    return correlate_box(src, fmt, X, Y, Z, k, w, mode, 0, 0, z0, X, Y, z1, T,
                         Aabs, nthreads);
}

int vkto_correlate_box(const void* src, int fmt, int64_t X, int64_t Y,
                       int64_t Z, int k, const double* w, int mode, int64_t x0,
                       int64_t y0, int64_t z0, int64_t x1, int64_t y1,
                       int64_t z1, double* T, double* Aabs, int nthreads)
{
    return correlate_box(src, fmt, X, Y, Z, k, w, mode, x0, y0, z0, x1, y1, z1,
                         T, Aabs, nthreads);
}

int vkto_correlate_points(const void* src, int fmt, int64_t X, int64_t Y,
                          int64_t Z, int k, const double* w, int mode,
                          const int64_t* pts, int64_t npts, double* T,
                          double* Aabs)
{
    if (check_filter_args(src, fmt, X, Y, Z, k, w, mode)) return -1;
    if (npts < 0 || (npts > 0 && (!pts || !T))) return -1;
    for (int64_t i = 0; i < npts; ++i) {
        int64_t x = pts[3 * i], y = pts[3 * i + 1], z = pts[3 * i + 2];
        if (x < 0 || y < 0 || z < 0 || x >= X || y >= Y || z >= Z) return -1;
        one_cell(src, fmt, X, Y, Z, k, w, mode, x, y, z, &T[i],
                 Aabs ? &Aabs[i] : NULL);
    }
    return 0;
}

/* ---- stored results ------------------------------------------------------ */

static double fmt_max(int fmt) { return fmt == VKTO_U8 ? 255.0 : 65535.0; }

static void store_int(void* out, int fmt, int64_t i, int64_t v)
{
    if (fmt == VKTO_U8) ((uint8_t*)out)[i] = (uint8_t)v;
    else ((uint16_t*)out)[i] = (uint16_t)v;
}

int vkto_store_float_filter(const double* q, int64_t n, int out_fmt, void* out)
{
    if ((n > 0 && (!q || !out)) || n < 0) return -1;
    for (int64_t i = 0; i < n; ++i) {
        if (out_fmt == VKTO_F32) {
            ((float*)out)[i] = (float)q[i];
        } else if (out_fmt == VKTO_U8 || out_fmt == VKTO_U16) {
            double v = floor(q[i] + 0.5);
            if (v < 0.0) v = 0.0;
            if (v > fmt_max(out_fmt)) v = fmt_max(out_fmt);
            store_int(out, out_fmt, i, (int64_t)v);
        } else {
            return -1;
        }
    }
    return 0;
}

/* floor(num / den) for den > 0, exact in integers */
static int64_t floor_div(int64_t num, int64_t den)
{
    int64_t q = num / den;
    if ((num % den) != 0 && num < 0) q -= 1;
    return q;
}

int vkto_store_int_filter(const double* T, int64_t n, int64_t D, int out_fmt,
                          void* out)
{
    if ((n > 0 && (!T || !out)) || n < 0 || D < 1) return -1;
    for (int64_t i = 0; i < n; ++i) {
        if (out_fmt == VKTO_F32) {
            ((float*)out)[i] = (float)(T[i] / (double)D);
        } else if (out_fmt == VKTO_U8 || out_fmt == VKTO_U16) {
            int64_t t = (int64_t)T[i]; /* T is an exact integer below 2^53 */
            int64_t v = floor_div(2 * t + D, 2 * D);
            int64_t mx = (int64_t)fmt_max(out_fmt);
            if (v < 0) v = 0;
            if (v > mx) v = mx;
            store_int(out, out_fmt, i, v);
        } else {
            return -1;
        }
    }
    return 0;
}

/* ---- Fill / FillRange ----------------------------------------------------- */

int vkto_fill_raw(double value, double lo, double hi, int fmt, double* raw)
{
    if (!raw) return -1;
    if (fmt == VKTO_F32) { *raw = (double)(float)value; return 0; }
    if (fmt != VKTO_U8 && fmt != VKTO_U16) return -1;
    if (hi == lo) return -1;
    double mx = fmt_max(fmt);
    double v = floor((value - lo) / (hi - lo) * mx + 0.5);
    if (v < 0.0) v = 0.0;
    if (v > mx) v = mx;
    *raw = v;
    return 0;
}

int vkto_fill_range(void* dst, int fmt, int64_t X, int64_t Y, int64_t Z,
                    int64_t x0, int64_t y0, int64_t z0, int64_t x1, int64_t y1,
                    int64_t z1, double raw)
{
    if (!dst || (fmt != VKTO_U8 && fmt != VKTO_U16 && fmt != VKTO_F32))
        return -1;
    if (x0 < 0 || y0 < 0 || z0 < 0 || x1 > X || y1 > Y || z1 > Z) return -1;
    if (x0 > x1 || y0 > y1 || z0 > z1) return -1;
    for (int64_t z = z0; z < z1; ++z)
        for (int64_t y = y0; y < y1; ++y)
            for (int64_t x = x0; x < x1; ++x) {
                int64_t i = x + X * (y + Y * z);
                if (fmt == VKTO_F32) ((float*)dst)[i] = (float)raw;
                else store_int(dst, fmt, i, (int64_t)raw);
            }
    return 0;
}

/* ---- Resample: trilinear, cell-centred, clamp to the volume (Sec. 3.2) --- */

/* Lower neighbour index and weight of the upper one for destination cell i
 * on an axis of n source and m destination cells. */
static void lin_axis(int64_t i, int64_t n, int64_t m, int64_t* i0, int64_t* i1, double* f)
{
    const double u = ((double)i + 0.5) * (double)n / (double)m - 0.5;
    const double fl = floor(u);
    int64_t a = (int64_t)fl, b = a + 1;
    *f = u - fl;
    if (a < 0) a = 0;
    if (a > n - 1) a = n - 1;
    if (b < 0) b = 0;
    if (b > n - 1) b = n - 1;
    *i0 = a;
    *i1 = b;
}

int vkto_resample_linear(const void* src, int fmt, int64_t X, int64_t Y, int64_t Z,
                         int64_t Xo, int64_t Yo, int64_t Zo, double* out, double* Aabs)
{
    if (!src || !out || !valid_fmt(fmt) || X < 1 || Y < 1 || Z < 1 || Xo < 1 || Yo < 1 ||
        Zo < 1)
        return -1;
    for (int64_t z = 0; z < Zo; ++z) {
        int64_t z0, z1;
        double fz;
        lin_axis(z, Z, Zo, &z0, &z1, &fz);
        for (int64_t y = 0; y < Yo; ++y) {
            int64_t y0, y1;
            double fy;
            lin_axis(y, Y, Yo, &y0, &y1, &fy);
            for (int64_t x = 0; x < Xo; ++x) {
                int64_t x0, x1;
                double fx;
                lin_axis(x, X, Xo, &x0, &x1, &fx);
                const int64_t xs[2] = {x0, x1}, ys[2] = {y0, y1}, zs[2] = {z0, z1};
                const double wx[2] = {1.0 - fx, fx}, wy[2] = {1.0 - fy, fy}, wz[2] = {1.0 - fz, fz};
                double s = 0.0, sa = 0.0;
                for (int c = 0; c < 2; ++c)
                    for (int b = 0; b < 2; ++b)
                        for (int a = 0; a < 2; ++a) {
                            const double w = wx[a] * wy[b] * wz[c];
                            const double v = load_cell(src, fmt, xs[a] + X * (ys[b] + Y * zs[c]));
                            s += w * v;
                            sa += fabs(w * v);
                        }
                const int64_t o = x + Xo * (y + Yo * z);
                out[o] = s;
                if (Aabs) Aabs[o] = sa;
            }
        }
    }
    return 0;
}

/* ---- Flip along one axis (Sec. 3.2 transform algorithms) ----------------- */

int vkto_flip(const void* src, int fmt, int64_t X, int64_t Y, int64_t Z, int axis, void* dst)
{
    if (!src || !dst || !valid_fmt(fmt) || X < 1 || Y < 1 || Z < 1 || axis < 0 || axis > 2)
        return -1;
    const size_t cb = fmt == VKTO_U8 ? 1 : fmt == VKTO_U16 ? 2 : fmt == VKTO_F32 ? 4 : 8;
    for (int64_t z = 0; z < Z; ++z)
        for (int64_t y = 0; y < Y; ++y)
            for (int64_t x = 0; x < X; ++x) {
                const int64_t sx = axis == 0 ? X - 1 - x : x;
                const int64_t sy = axis == 1 ? Y - 1 - y : y;
                const int64_t sz = axis == 2 ? Z - 1 - z : z;
                memcpy((char*)dst + (x + X * (y + Y * z)) * cb,
                       (const char*)src + (sx + X * (sy + Y * sz)) * cb, cb);
            }
    return 0;
}

/* ---- BrickDecompose: one brick with ghost cells (Sec. 3.2) --------------- */

int vkto_brick(const void* src, int fmt, int64_t X, int64_t Y, int64_t Z, int64_t x0,
               int64_t y0, int64_t z0, int64_t nx, int64_t ny, int64_t nz, int mode,
               void* dst)
{
    if (!src || !dst || !valid_fmt(fmt) || X < 1 || Y < 1 || Z < 1 || nx < 0 || ny < 0 ||
        nz < 0 || mode < VKTO_CLAMP || mode > VKTO_BORDER)
        return -1;
    const size_t cb = fmt == VKTO_U8 ? 1 : fmt == VKTO_U16 ? 2 : fmt == VKTO_F32 ? 4 : 8;
    for (int64_t k = 0; k < nz; ++k)
        for (int64_t j = 0; j < ny; ++j)
            for (int64_t i = 0; i < nx; ++i) {
                char* out = (char*)dst + (i + nx * (j + ny * k)) * cb;
                const int64_t sx = vkto_address(x0 + i, X, mode);
                const int64_t sy = vkto_address(y0 + j, Y, mode);
                const int64_t sz = vkto_address(z0 + k, Z, mode);
                if (sx < 0 || sy < 0 || sz < 0)
                    memset(out, 0, cb);
                else
                    memcpy(out, (const char*)src + (sx + X * (sy + Y * sz)) * cb, cb);
            }
    return 0;
}
