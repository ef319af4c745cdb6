"""Python binding of libvkt (include/vkt.h): argument marshalling only.

Every call goes through the C interface of the in-tree libvkt.so; all volume
arithmetic runs in its HIP kernels.  torch supplies device memory (tensors)
and streams.  There is no fallback: if libvkt.so is missing, or no GPU is
visible when a call needs one, the call raises.

The function names are the C names.  Handles are opaque integers.
"""
import ctypes
import os

import torch  # loads torch's HIP runtime first; libvkt then binds to it

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvkt.so")

# enums of include/vkt.h
vktNoError, vktInvalidValue, vktOutOfMemory, vktDeviceError, vktUnsupported = range(5)
vktDataFormatUInt8, vktDataFormatUInt16, vktDataFormatFloat32 = range(3)
vktAddressModeClamp, vktAddressModeWrap, vktAddressModeMirror, vktAddressModeBorder = range(4)
vktPrecisionAuto, vktPrecisionFP32, vktPrecisionSplitBF16, vktPrecisionSplitBF16x6 = range(4)
vktAxisX, vktAxisY, vktAxisZ = range(3)
(vktFilterPathVectorFP32, vktFilterPathDot8, vktFilterPathInt8Matrix,
 vktFilterPathSplitMatrix, vktFilterPathSeparable) = range(5)
FILTER_PATHS = {vktFilterPathVectorFP32: "valu", vktFilterPathDot8: "dot4",
                vktFilterPathInt8Matrix: "i8mma", vktFilterPathSplitMatrix: "mfma",
                vktFilterPathSeparable: "sep"}

MODES = {"clamp": vktAddressModeClamp, "wrap": vktAddressModeWrap,
         "mirror": vktAddressModeMirror, "border": vktAddressModeBorder}
PRECISIONS = {"auto": vktPrecisionAuto, "fp32": vktPrecisionFP32,
              "splitbf16": vktPrecisionSplitBF16, "splitbf16x6": vktPrecisionSplitBF16x6}
TORCH_FORMAT = {torch.uint8: vktDataFormatUInt8, torch.uint16: vktDataFormatUInt16,
                torch.float32: vktDataFormatFloat32}

# Every function include/vkt.h declares, with its argument types.
_P, _I32, _F = ctypes.c_void_p, ctypes.c_int32, ctypes.c_float
_PP = ctypes.POINTER(ctypes.c_void_p)
_PI = ctypes.POINTER(ctypes.c_int32)
SIGNATURES = {
    "vktStructuredVolumeCreate": [_PP, _I32, _I32, _I32, ctypes.c_int, _F, _F, _F, _F, _F],
    "vktStructuredVolumeCreateFromDevicePtr": [_PP, _I32, _I32, _I32, ctypes.c_int, _P, _F, _F],
    "vktStructuredVolumeDestroy": [_P],
    "vktStructuredVolumeGetDevicePtr": [_P, _PP],
    "vktStructuredVolumeGetDims": [_P, _PI, _PI, _PI],
    "vktStructuredVolumeGetDataFormat": [_P, ctypes.POINTER(ctypes.c_int)],
    "vktFilterCreate": [_PP, _I32, ctypes.POINTER(ctypes.c_float)],
    "vktFilterCreateInt": [_PP, _I32, _PI, _I32],
    "vktFilterDestroy": [_P],
    "vktFill": [_P, _F],
    "vktFillRange": [_P, _I32, _I32, _I32, _I32, _I32, _I32, _F],
    "vktFillSV": [_P, _F],
    "vktFillRangeSV": [_P, _I32, _I32, _I32, _I32, _I32, _I32, _F],
    "vktApplyFilter": [_P, _P, _P, ctypes.c_int],
    "vktApplyFilterRange": [_P, _P, _P, _I32, _I32, _I32, _I32, _I32, _I32, ctypes.c_int],
    "vktApplyFilterBatched": [_I32, _PP, _PP, _PP, ctypes.c_int],
    "vktApplyFilterBatchedNoAlloc": [_I32, _PP, _PP, _PP, ctypes.c_int],
    "vktBrickDecomposeGetNumBricks": [_P, _I32, _I32, _I32, _PI, _PI, _PI],
    "vktBrickDecomposeGetBrickDims": [_P, _I32, _I32, _I32, _I32, _I32, _I32, _I32, _I32, _I32,
                                      _PI, _PI, _PI],
    "vktBrickDecompose": [_I32, _PP, _P, _I32, _I32, _I32, _I32, _I32, _I32, ctypes.c_int],
    "vktBrickDecomposeSV": [_I32, _PP, _P, _I32, _I32, _I32, _I32, _I32, _I32, ctypes.c_int],
    "vktResample": [_P, _P],
    "vktFlip": [_P, _P, ctypes.c_int],
    "vktResampleSV": [_P, _P],
    "vktFlipSV": [_P, _P, ctypes.c_int],
    "vktSetAutotune": [ctypes.c_int],
    "vktSetSeparable": [ctypes.c_int],
    "vktGetSeparable": [ctypes.POINTER(ctypes.c_int)],
    "vktSetInt8Matrix": [ctypes.c_int],
    "vktGetInt8Matrix": [ctypes.POINTER(ctypes.c_int)],
    "vktSetRowPairMinCells": [ctypes.c_int64],
    "vktGetRowPairMinCells": [ctypes.POINTER(ctypes.c_int64)],
    "vktFilterIsSeparable": [_P, ctypes.POINTER(ctypes.c_int)],
    "vktGetFilterPath": [_P, _P, _P, ctypes.c_int, ctypes.POINTER(ctypes.c_int), _PI],
    "vktSetStream": [_P],
    "vktGetStream": [_PP],
    "vktSetPrecision": [ctypes.c_int],
    "vktGetPrecision": [ctypes.POINTER(ctypes.c_int)],
    "vktSynchronize": [],
    "vktGetErrorString": [ctypes.c_int],
}


class VktError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        super().__init__(f"{where}: {error_string(code)} ({code})")


_lib = None


def lib():
    """Load the in-tree libvkt.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, args in SIGNATURES.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_char_p if name == "vktGetErrorString" else ctypes.c_int
        _lib = L
    return _lib


def error_string(code):
    return lib().vktGetErrorString(int(code)).decode()


def _ok(code, where):
    if code != vktNoError:
        raise VktError(code, where)


def _require_gpu():
    if not torch.cuda.is_available():
        raise RuntimeError("libvkt needs a visible GPU; none is available")


# ------------------------------------------------------------------ volumes --

def vktStructuredVolumeCreate(dims, fmt, cell=(1.0, 1.0, 1.0), lo=0.0, hi=1.0):
    """Owned, zero-filled device volume; dims = (X, Y, Z)."""
    _require_gpu()
    h = ctypes.c_void_p()
    _ok(lib().vktStructuredVolumeCreate(ctypes.byref(h), *[int(d) for d in dims],
                                        int(fmt), *[float(c) for c in cell],
                                        float(lo), float(hi)),
        "vktStructuredVolumeCreate")
    return h.value


def vktStructuredVolumeCreateFromDevicePtr(dims, fmt, ptr, lo=0.0, hi=1.0):
    h = ctypes.c_void_p()
    _ok(lib().vktStructuredVolumeCreateFromDevicePtr(
        ctypes.byref(h), *[int(d) for d in dims], int(fmt), ctypes.c_void_p(ptr),
        float(lo), float(hi)), "vktStructuredVolumeCreateFromDevicePtr")
    return h.value


def vktStructuredVolumeDestroy(h):
    _ok(lib().vktStructuredVolumeDestroy(h), "vktStructuredVolumeDestroy")


def vktStructuredVolumeGetDevicePtr(h):
    p = ctypes.c_void_p()
    _ok(lib().vktStructuredVolumeGetDevicePtr(h, ctypes.byref(p)),
        "vktStructuredVolumeGetDevicePtr")
    return p.value


def vktStructuredVolumeGetDims(h):
    d = [ctypes.c_int32() for _ in range(3)]
    _ok(lib().vktStructuredVolumeGetDims(h, *[ctypes.byref(v) for v in d]),
        "vktStructuredVolumeGetDims")
    return tuple(v.value for v in d)


def vktStructuredVolumeGetDataFormat(h):
    f = ctypes.c_int()
    _ok(lib().vktStructuredVolumeGetDataFormat(h, ctypes.byref(f)),
        "vktStructuredVolumeGetDataFormat")
    return f.value


# ------------------------------------------------------------------ filters --

def vktFilterCreate(weights):
    """weights: (k, k, k) array-like indexed [c, b, a]; copied as float32."""
    import numpy as np
    w = np.ascontiguousarray(weights, dtype=np.float32)
    k = w.shape[0]
    if w.shape != (k, k, k):
        raise ValueError("filter must be k*k*k")
    h = ctypes.c_void_p()
    _ok(lib().vktFilterCreate(ctypes.byref(h), k,
                              w.ctypes.data_as(ctypes.POINTER(ctypes.c_float))),
        "vktFilterCreate")
    return h.value


def vktFilterCreateInt(weights, divisor):
    import numpy as np
    w = np.ascontiguousarray(weights, dtype=np.int32)
    k = w.shape[0]
    if w.shape != (k, k, k):
        raise ValueError("filter must be k*k*k")
    h = ctypes.c_void_p()
    _ok(lib().vktFilterCreateInt(ctypes.byref(h), k,
                                 w.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                 int(divisor)), "vktFilterCreateInt")
    return h.value


def vktFilterDestroy(h):
    _ok(lib().vktFilterDestroy(h), "vktFilterDestroy")


# ------------------------------------------------------------- algorithms --

def vktFill(vol, value):
    _ok(lib().vktFill(vol, float(value)), "vktFill")


def vktFillRange(vol, first, last, value):
    _ok(lib().vktFillRange(vol, *[int(v) for v in first], *[int(v) for v in last],
                           float(value)), "vktFillRange")


vktFillSV = vktFill
vktFillRangeSV = vktFillRange


def vktApplyFilter(dst, src, filt, mode=vktAddressModeClamp):
    m = MODES[mode] if isinstance(mode, str) else int(mode)
    _ok(lib().vktApplyFilter(dst, src, filt, m), "vktApplyFilter")


def vktApplyFilterRange(dst, src, filt, first, last, mode=vktAddressModeClamp):
    """first, last: (x, y, z) bounds of the half-open output region."""
    m = MODES[mode] if isinstance(mode, str) else int(mode)
    _ok(lib().vktApplyFilterRange(dst, src, filt, *[int(v) for v in first],
                                  *[int(v) for v in last], m), "vktApplyFilterRange")


def vktApplyFilterBatched(dsts, srcs, filts, mode=vktAddressModeClamp):
    """dsts, srcs, filts: equal-length sequences of handles."""
    n = len(dsts)
    if len(srcs) != n or len(filts) != n:
        raise ValueError("batched call needs equal-length handle lists")
    arr = ctypes.c_void_p * max(n, 1)
    m = MODES[mode] if isinstance(mode, str) else int(mode)
    _ok(lib().vktApplyFilterBatched(n, arr(*dsts), arr(*srcs), arr(*filts), m),
        "vktApplyFilterBatched")


def vktApplyFilterBatchedNoAlloc(dsts, srcs, filts, mode=vktAddressModeClamp):
    """As vktApplyFilterBatched, with no device allocation (static scratch)."""
    n = len(dsts)
    if len(srcs) != n or len(filts) != n:
        raise ValueError("batched call needs equal-length handle lists")
    arr = ctypes.c_void_p * max(n, 1)
    m = MODES[mode] if isinstance(mode, str) else int(mode)
    _ok(lib().vktApplyFilterBatchedNoAlloc(n, arr(*dsts), arr(*srcs), arr(*filts), m),
        "vktApplyFilterBatchedNoAlloc")


def vktResample(dst, src):
    _ok(lib().vktResample(dst, src), "vktResample")


def vktFlip(dst, src, axis):
    """axis: 0 / vktAxisX, 1 / vktAxisY, 2 / vktAxisZ; dst == src flips in place."""
    _ok(lib().vktFlip(dst, src, int(axis)), "vktFlip")


def vktBrickDecomposeGetNumBricks(src, brick):
    """brick = (x, y, z) interior cells; returns bricks per axis (x, y, z)."""
    n = [ctypes.c_int32() for _ in range(3)]
    _ok(lib().vktBrickDecomposeGetNumBricks(src, *[int(b) for b in brick],
                                            *[ctypes.byref(v) for v in n]),
        "vktBrickDecomposeGetNumBricks")
    return tuple(v.value for v in n)


def vktBrickDecomposeGetBrickDims(src, brick, ghost, index):
    """Dims (x, y, z) of brick index = (bx, by, bz), ghosts included."""
    d = [ctypes.c_int32() for _ in range(3)]
    _ok(lib().vktBrickDecomposeGetBrickDims(src, *[int(b) for b in brick],
                                            *[int(g) for g in ghost], *[int(i) for i in index],
                                            *[ctypes.byref(v) for v in d]),
        "vktBrickDecomposeGetBrickDims")
    return tuple(v.value for v in d)


def vktBrickDecompose(bricks, src, brick, ghost=(0, 0, 0), mode=vktAddressModeClamp):
    """bricks: handles in order bx + numX * (by + numY * bz)."""
    n = len(bricks)
    arr = ctypes.c_void_p * max(n, 1)
    m = MODES[mode] if isinstance(mode, str) else int(mode)
    _ok(lib().vktBrickDecompose(n, arr(*bricks), src, *[int(b) for b in brick],
                                *[int(g) for g in ghost], m), "vktBrickDecompose")


vktBrickDecomposeSV = vktBrickDecompose
vktResampleSV = vktResample
vktFlipSV = vktFlip


# ------------------------------------------------------------- thread state --

def vktSetStream(stream):
    """stream: a torch.cuda.Stream, a raw hipStream_t integer, or None."""
    if isinstance(stream, torch.cuda.Stream):
        stream = stream.cuda_stream
    _ok(lib().vktSetStream(ctypes.c_void_p(stream or None)), "vktSetStream")


def vktGetStream():
    p = ctypes.c_void_p()
    _ok(lib().vktGetStream(ctypes.byref(p)), "vktGetStream")
    return p.value


def vktSetPrecision(p):
    p = PRECISIONS[p] if isinstance(p, str) else int(p)
    _ok(lib().vktSetPrecision(p), "vktSetPrecision")


def vktGetPrecision():
    p = ctypes.c_int()
    _ok(lib().vktGetPrecision(ctypes.byref(p)), "vktGetPrecision")
    return p.value


def vktSetAutotune(enable):
    _ok(lib().vktSetAutotune(1 if enable else 0), "vktSetAutotune")


def vktSetSeparable(enable):
    _ok(lib().vktSetSeparable(1 if enable else 0), "vktSetSeparable")


def vktGetSeparable():
    v = ctypes.c_int()
    _ok(lib().vktGetSeparable(ctypes.byref(v)), "vktGetSeparable")
    return bool(v.value)


def vktSetInt8Matrix(enable):
    _ok(lib().vktSetInt8Matrix(1 if enable else 0), "vktSetInt8Matrix")


def vktGetInt8Matrix():
    v = ctypes.c_int()
    _ok(lib().vktGetInt8Matrix(ctypes.byref(v)), "vktGetInt8Matrix")
    return bool(v.value)


def vktSetRowPairMinCells(cells):
    _ok(lib().vktSetRowPairMinCells(int(cells)), "vktSetRowPairMinCells")


def vktGetRowPairMinCells():
    v = ctypes.c_int64()
    _ok(lib().vktGetRowPairMinCells(ctypes.byref(v)), "vktGetRowPairMinCells")
    return v.value


def vktFilterIsSeparable(filt):
    v = ctypes.c_int()
    _ok(lib().vktFilterIsSeparable(filt, ctypes.byref(v)), "vktFilterIsSeparable")
    return bool(v.value)


def vktGetFilterPath(dst, src, filt, mode=vktAddressModeClamp):
    """(path, products) that vktApplyFilter(dst, src, filt, mode) would take
    on this thread now; path is a vktFilterPath value."""
    m = MODES[mode] if isinstance(mode, str) else int(mode)
    p = ctypes.c_int()
    n = ctypes.c_int32()
    _ok(lib().vktGetFilterPath(dst, src, filt, m, ctypes.byref(p), ctypes.byref(n)),
        "vktGetFilterPath")
    return p.value, n.value


def vktSynchronize():
    _ok(lib().vktSynchronize(), "vktSynchronize")


# ------------------------------------------------------ tensor conveniences --

def volume_from_tensor(t, lo=0.0, hi=1.0):
    """Borrowing handle for a contiguous (Z, Y, X) device tensor."""
    if not t.is_cuda or not t.is_contiguous() or t.dim() != 3:
        raise ValueError("need a contiguous 3-D device tensor")
    if t.dtype not in TORCH_FORMAT:
        raise ValueError(f"unsupported dtype {t.dtype}")
    Z, Y, X = t.shape
    return vktStructuredVolumeCreateFromDevicePtr((X, Y, Z), TORCH_FORMAT[t.dtype],
                                                  t.data_ptr(), lo, hi)


def apply_filter(dst, src, weights, mode="clamp", divisor=None, roi=None):
    """One ApplyFilter of src into dst (device tensors) on torch's current
    stream; integer weights with `divisor` create an integer filter; roi =
    ((x0, y0, z0), (x1, y1, z1)) runs the range version."""
    vktSetStream(torch.cuda.current_stream())
    hs = volume_from_tensor(src)
    hd = volume_from_tensor(dst)
    hf = vktFilterCreate(weights) if divisor is None else vktFilterCreateInt(weights, divisor)
    try:
        if roi is None:
            vktApplyFilter(hd, hs, hf, mode)
        else:
            vktApplyFilterRange(hd, hs, hf, roi[0], roi[1], mode)
    finally:
        vktFilterDestroy(hf)
        vktStructuredVolumeDestroy(hd)
        vktStructuredVolumeDestroy(hs)


def resample(dst, src):
    """Resample device tensor src onto dst's shape on torch's current stream."""
    vktSetStream(torch.cuda.current_stream())
    hs = volume_from_tensor(src)
    hd = volume_from_tensor(dst)
    try:
        vktResample(hd, hs)
    finally:
        vktStructuredVolumeDestroy(hd)
        vktStructuredVolumeDestroy(hs)


def flip(dst, src, axis):
    """Flip device tensor src into dst (dst may be src) along axis 0 = x,
    1 = y, 2 = z on torch's current stream."""
    vktSetStream(torch.cuda.current_stream())
    hs = volume_from_tensor(src)
    hd = volume_from_tensor(dst)
    try:
        vktFlip(hd, hs, axis)
    finally:
        vktStructuredVolumeDestroy(hd)
        vktStructuredVolumeDestroy(hs)


def brick_decompose(src, brick, ghost=(0, 0, 0), mode="clamp"):
    """Bricks of device tensor src (Z, Y, X) as new device tensors, in order
    bx + numX * (by + numY * bz), on torch's current stream."""
    vktSetStream(torch.cuda.current_stream())
    hs = volume_from_tensor(src)
    out, hb = [], []
    try:
        nx, ny, nz = vktBrickDecomposeGetNumBricks(hs, brick)
        for bz in range(nz):
            for by in range(ny):
                for bx in range(nx):
                    dx, dy, dz = vktBrickDecomposeGetBrickDims(hs, brick, ghost, (bx, by, bz))
                    t = torch.empty((dz, dy, dx), dtype=src.dtype, device=src.device)
                    out.append(t)
                    hb.append(volume_from_tensor(t))
        vktBrickDecompose(hb, hs, brick, ghost, mode)
    finally:
        for h in hb:
            vktStructuredVolumeDestroy(h)
        vktStructuredVolumeDestroy(hs)
    return out
