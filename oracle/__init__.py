"""FP64 host oracle for volkit's ApplyFilter / Fill / FillRange (ctypes front).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark may import this package; the GPU library and its Python
binding never do.

Arrays follow the volume layout of the paper's structured volumes with x the
fastest axis, so a numpy volume has shape (Z, Y, X) and a filter has shape
(k, k, k) indexed [c, b, a] (tap (a, b, c) reads src(x+a-r, y+b-r, z+c-r)).
"""
import ctypes
import os

import numpy as np

from ._build import LIB, build_oracle

__all__ = ["MODES", "correlate", "correlate_box", "correlate_points", "store_float_filter",
           "store_int_filter", "apply_filter", "fill_raw", "fill_range",
           "address", "resample", "flip", "brick_grid", "brick_decompose", "lib"]

MODES = {"clamp": 0, "wrap": 1, "mirror": 2, "border": 3}
_FMT = {np.dtype(np.uint8): 0, np.dtype(np.uint16): 1,
        np.dtype(np.float32): 2, np.dtype(np.float64): 3}

_lib = None


def lib():
    """Load libvkt_oracle.so, compiling it first if it is not built yet."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB):
        build_oracle()
    L = ctypes.CDLL(LIB)
    i64, dp, vp = ctypes.c_int64, ctypes.POINTER(ctypes.c_double), ctypes.c_void_p
    L.vkto_address.argtypes = [i64, i64, ctypes.c_int]
    L.vkto_address.restype = i64
    L.vkto_correlate.argtypes = [vp, ctypes.c_int, i64, i64, i64, ctypes.c_int,
                                 dp, ctypes.c_int, i64, i64, dp, dp, ctypes.c_int]
    L.vkto_correlate_box.argtypes = [vp, ctypes.c_int, i64, i64, i64, ctypes.c_int,
                                     dp, ctypes.c_int, i64, i64, i64, i64, i64, i64,
                                     dp, dp, ctypes.c_int]
    L.vkto_correlate_points.argtypes = [vp, ctypes.c_int, i64, i64, i64,
                                        ctypes.c_int, dp, ctypes.c_int,
                                        ctypes.POINTER(i64), i64, dp, dp]
    L.vkto_store_float_filter.argtypes = [dp, i64, ctypes.c_int, vp]
    L.vkto_store_int_filter.argtypes = [dp, i64, i64, ctypes.c_int, vp]
    L.vkto_fill_raw.argtypes = [ctypes.c_double, ctypes.c_double,
                                ctypes.c_double, ctypes.c_int, dp]
    L.vkto_fill_range.argtypes = [vp, ctypes.c_int, i64, i64, i64, i64, i64,
                                  i64, i64, i64, i64, ctypes.c_double]
    L.vkto_resample_linear.argtypes = [vp, ctypes.c_int, i64, i64, i64, i64, i64, i64,
                                       dp, dp]
    L.vkto_flip.argtypes = [vp, ctypes.c_int, i64, i64, i64, ctypes.c_int, vp]
    L.vkto_brick.argtypes = [vp, ctypes.c_int, i64, i64, i64, i64, i64, i64, i64, i64, i64,
                             ctypes.c_int, vp]
    for f in ("vkto_correlate", "vkto_correlate_box", "vkto_correlate_points",
              "vkto_store_float_filter", "vkto_store_int_filter",
              "vkto_fill_raw", "vkto_fill_range", "vkto_resample_linear", "vkto_flip",
              "vkto_brick"):
        getattr(L, f).restype = ctypes.c_int
    _lib = L
    return L


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _mode(mode):
    return MODES[mode] if isinstance(mode, str) else int(mode)


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what}: bad argument (rc={rc})")


def _volume(src):
    src = np.ascontiguousarray(src)
    if src.ndim != 3 or src.dtype not in _FMT:
        raise ValueError("volume must be a 3-D uint8/uint16/float32/float64 array")
    return src


def _filter(w):
    w = np.ascontiguousarray(w, dtype=np.float64)
    k = w.shape[0]
    if w.shape != (k, k, k):
        raise ValueError("filter must be k*k*k")
    return w, k


def address(i, n, mode):
    return int(lib().vkto_address(int(i), int(n), _mode(mode)))


def correlate(src, w, mode="clamp", z_range=None, nthreads=0, with_abs=True):
    """T (and A_abs = sum |w||s|) at every cell, FP64; shape (nz, Y, X)."""
    src = _volume(src)
    w, k = _filter(w)
    Z, Y, X = src.shape
    z0, z1 = (0, Z) if z_range is None else z_range
    T = np.empty((z1 - z0, Y, X), np.float64)
    A = np.empty_like(T) if with_abs else None
    rc = lib().vkto_correlate(src.ctypes.data, _FMT[src.dtype], X, Y, Z, k,
                              _dp(w), _mode(mode), z0, z1, _dp(T),
                              _dp(A) if with_abs else None, int(nthreads))
    _check(rc, "correlate")
    return (T, A) if with_abs else T


def correlate_box(src, w, mode, first, last, nthreads=0, with_abs=True):
    """T (and A_abs) on the half-open box [first, last), first/last = (x, y,
    z), read through the address mode at the volume's faces; shape (nz, ny,
    nx)."""
    src = _volume(src)
    w, k = _filter(w)
    Z, Y, X = src.shape
    (x0, y0, z0), (x1, y1, z1) = first, last
    T = np.empty((max(z1 - z0, 0), max(y1 - y0, 0), max(x1 - x0, 0)), np.float64)
    A = np.empty_like(T) if with_abs else None
    rc = lib().vkto_correlate_box(src.ctypes.data, _FMT[src.dtype], X, Y, Z, k,
                                  _dp(w), _mode(mode), int(x0), int(y0), int(z0),
                                  int(x1), int(y1), int(z1), _dp(T),
                                  _dp(A) if with_abs else None, int(nthreads))
    _check(rc, "correlate_box")
    return (T, A) if with_abs else T


def correlate_points(src, w, mode, pts):
    """T and A_abs at the cells pts[i] = (x, y, z)."""
    src = _volume(src)
    w, k = _filter(w)
    Z, Y, X = src.shape
    pts = np.ascontiguousarray(pts, dtype=np.int64).reshape(-1, 3)
    n = pts.shape[0]
    T = np.empty(n, np.float64)
    A = np.empty(n, np.float64)
    rc = lib().vkto_correlate_points(
        src.ctypes.data, _FMT[src.dtype], X, Y, Z, k, _dp(w), _mode(mode),
        pts.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), n, _dp(T), _dp(A))
    _check(rc, "correlate_points")
    return T, A


def store_float_filter(q, out_dtype):
    q = np.ascontiguousarray(q, dtype=np.float64)
    out = np.empty(q.shape, out_dtype)
    _check(lib().vkto_store_float_filter(_dp(q), q.size, _FMT[out.dtype],
                                         out.ctypes.data), "store_float_filter")
    return out


def store_int_filter(T, divisor, out_dtype):
    T = np.ascontiguousarray(T, dtype=np.float64)
    out = np.empty(T.shape, out_dtype)
    _check(lib().vkto_store_int_filter(_dp(T), T.size, int(divisor),
                                       _FMT[out.dtype], out.ctypes.data),
           "store_int_filter")
    return out


def apply_filter(src, w, mode="clamp", divisor=None, z_range=None, nthreads=0):
    """Stored ApplyFilter result in src's format.

    Float weights (divisor None): q = T.  Integer weights: T / divisor with
    the exact half-up integer rounding."""
    T = correlate(src, w, mode, z_range, nthreads, with_abs=False)
    if divisor is None:
        return store_float_filter(T, src.dtype)
    return store_int_filter(T, divisor, src.dtype)


def fill_raw(value, lo, hi, dtype):
    raw = ctypes.c_double()
    _check(lib().vkto_fill_raw(float(value), float(lo), float(hi),
                               _FMT[np.dtype(dtype)], ctypes.byref(raw)),
           "fill_raw")
    return raw.value


def fill_range(vol, first, last, raw):
    """In place: cells of the half-open box [first, last) (x, y, z) := raw."""
    if not vol.flags.c_contiguous:
        raise ValueError("volume must be contiguous")
    Z, Y, X = vol.shape
    _check(lib().vkto_fill_range(vol.ctypes.data, _FMT[vol.dtype], X, Y, Z,
                                 *[int(v) for v in first],
                                 *[int(v) for v in last], float(raw)),
           "fill_range")
    return vol


def resample(src, dims):
    """Trilinear cell-centred resampling of src (Z, Y, X) to dims = (X, Y, Z)
    (paper Sec. 3.2 Resample); returns (values, sum of |w s|) in FP64."""
    src = _volume(src)
    Xo, Yo, Zo = (int(d) for d in dims)
    Z, Y, X = src.shape
    out = np.empty((Zo, Yo, Xo), np.float64)
    A = np.empty_like(out)
    _check(lib().vkto_resample_linear(src.ctypes.data, _FMT[src.dtype], X, Y, Z, Xo, Yo, Zo,
                                      _dp(out), _dp(A)), "vkto_resample_linear")
    return out, A


def flip(src, axis):
    """src mirrored along axis 0 = x, 1 = y, 2 = z (paper Sec. 3.2 Flip)."""
    src = _volume(src)
    Z, Y, X = src.shape
    out = np.empty_like(src)
    _check(lib().vkto_flip(src.ctypes.data, _FMT[src.dtype], X, Y, Z, int(axis),
                           out.ctypes.data), "vkto_flip")
    return out


def brick_grid(dims, brick):
    """Bricks per axis: ceil(dim / brick) for dims, brick = (x, y, z)."""
    return tuple(-(-int(d) // int(b)) for d, b in zip(dims, brick))


def brick_decompose(src, brick, ghost=(0, 0, 0), mode="clamp"):
    """Split src (Z, Y, X) into bricks of brick = (BX, BY, BZ) interior cells
    (the last brick on an axis keeps the remainder), each with ghost =
    (gx, gy, gz) extra cells on both sides read through the address mode
    (paper Sec. 3.2 BrickDecompose).  Returns the bricks in order of brick
    index bx + nbx * (by + nby * bz), each a (Z, Y, X) array."""
    src = _volume(src)
    Z, Y, X = src.shape
    m = MODES[mode] if isinstance(mode, str) else int(mode)
    (BX, BY, BZ), (gx, gy, gz) = brick, ghost
    nbx, nby, nbz = brick_grid((X, Y, Z), brick)
    out = []
    for bz in range(nbz):
        for by in range(nby):
            for bx in range(nbx):
                ix = min(BX, X - bx * BX)
                iy = min(BY, Y - by * BY)
                iz = min(BZ, Z - bz * BZ)
                b = np.empty((iz + 2 * gz, iy + 2 * gy, ix + 2 * gx), src.dtype)
                _check(lib().vkto_brick(src.ctypes.data, _FMT[src.dtype], X, Y, Z,
                                        bx * BX - gx, by * BY - gy, bz * BZ - gz,
                                        ix + 2 * gx, iy + 2 * gy, iz + 2 * gz, m,
                                        b.ctypes.data), "vkto_brick")
                out.append(b)
    return out
