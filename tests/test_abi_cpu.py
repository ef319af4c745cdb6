"""Host-only checks of the C interface: the library loads, exports every
function include/vkt.h declares, and rejects bad arguments before it touches
the GPU.  No compute call is made here."""
import os
import re
import threading

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "vkt.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(vkt[A-Za-z0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def vkt():
    from paper_2203_10213_amd import vkt as v
    v.lib()
    return v


def test_every_declared_symbol_is_exported(vkt):
    names = declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(vkt.lib(), n), n
    # the binding declares exactly the header's functions
    assert sorted(vkt.SIGNATURES) == names


def test_error_strings(vkt):
    assert vkt.error_string(vkt.vktNoError) == "no error"
    assert vkt.error_string(vkt.vktInvalidValue) == "invalid value"
    assert vkt.error_string(vkt.vktUnsupported) == "unsupported"
    assert vkt.error_string(99) == "unknown error"


def test_null_handles_rejected_without_gpu(vkt):
    L = vkt.lib()
    assert L.vktApplyFilter(None, None, None, 0) == vkt.vktInvalidValue
    assert L.vktApplyFilterRange(None, None, None, 0, 0, 0, 1, 1, 1, 0) == vkt.vktInvalidValue
    assert L.vktFill(None, 1.0) == vkt.vktInvalidValue
    assert L.vktFillRange(None, 0, 0, 0, 1, 1, 1, 1.0) == vkt.vktInvalidValue
    assert L.vktFilterDestroy(None) == vkt.vktInvalidValue
    assert L.vktStructuredVolumeDestroy(None) == vkt.vktInvalidValue
    assert L.vktStructuredVolumeGetDevicePtr(None, None) == vkt.vktInvalidValue
    # a pointer that was never a handle is rejected, not dereferenced
    bogus = 0x1000
    assert L.vktApplyFilter(bogus, bogus, bogus, 0) == vkt.vktInvalidValue
    assert L.vktApplyFilterRange(bogus, bogus, bogus, 0, 0, 0, 1, 1, 1, 0) == vkt.vktInvalidValue
    for f in (L.vktResample, L.vktResampleSV):
        assert f(None, None) == vkt.vktInvalidValue
        assert f(bogus, bogus) == vkt.vktInvalidValue
    for f in (L.vktFlip, L.vktFlipSV):
        assert f(None, None, 0) == vkt.vktInvalidValue
        assert f(bogus, bogus, 1) == vkt.vktInvalidValue
    assert L.vktBrickDecompose(0, None, None, 1, 1, 1, 0, 0, 0, 0) == vkt.vktInvalidValue
    assert L.vktBrickDecomposeSV(1, None, bogus, 1, 1, 1, 0, 0, 0, 0) == vkt.vktInvalidValue
    assert L.vktBrickDecomposeGetNumBricks(bogus, 1, 1, 1, None, None, None) \
        == vkt.vktInvalidValue
    assert L.vktBrickDecomposeGetBrickDims(None, 1, 1, 1, 0, 0, 0, 0, 0, 0, None, None, None) \
        == vkt.vktInvalidValue
    # bad k / NULL weights fail before any device allocation
    assert L.vktFilterCreate(None, 3, None) == vkt.vktInvalidValue
    assert L.vktStructuredVolumeCreate(None, 4, 4, 4, 0, 1, 1, 1, 0, 1) == vkt.vktInvalidValue
    assert L.vktStructuredVolumeCreateFromDevicePtr(None, 4, 4, 4, 0, None, 0, 1) \
        == vkt.vktInvalidValue
    assert L.vktGetInt8Matrix(None) == vkt.vktInvalidValue
    assert L.vktGetSeparable(None) == vkt.vktInvalidValue


def test_filter_validation_without_gpu(vkt):
    import ctypes
    import numpy as np
    L = vkt.lib()
    h = ctypes.c_void_p()
    w = np.ones(16 ** 3, np.float32)
    wp = w.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    for k in (0, 2, 4, 16, 17, -1):
        assert L.vktFilterCreate(ctypes.byref(h), k, wp) == vkt.vktInvalidValue
    wi = np.ones(27, np.int32)
    wip = wi.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    assert L.vktFilterCreateInt(ctypes.byref(h), 3, wip, 0) == vkt.vktInvalidValue
    assert L.vktFilterCreateInt(ctypes.byref(h), 3, wip, (1 << 29) + 1) == vkt.vktInvalidValue
    wi[5] = 1 << 23
    assert L.vktFilterCreateInt(ctypes.byref(h), 3, wip, 1) == vkt.vktInvalidValue


def test_precision_is_thread_local(vkt):
    vkt.vktSetPrecision("splitbf16")
    seen = {}

    def other():
        seen["p"] = vkt.vktGetPrecision()
        vkt.vktSetPrecision("fp32")
        seen["q"] = vkt.vktGetPrecision()

    th = threading.Thread(target=other)
    th.start()
    th.join()
    assert seen == {"p": vkt.vktPrecisionAuto, "q": vkt.vktPrecisionFP32}
    assert vkt.vktGetPrecision() == vkt.vktPrecisionSplitBF16
    assert vkt.lib().vktSetPrecision(7) == vkt.vktInvalidValue
    vkt.vktSetPrecision("auto")


def test_int8_matrix_switch_is_thread_local(vkt):
    assert vkt.vktGetInt8Matrix() is False  # opt-in
    vkt.vktSetInt8Matrix(True)
    seen = {}

    def other():
        seen["p"] = vkt.vktGetInt8Matrix()

    th = threading.Thread(target=other)
    th.start()
    th.join()
    assert seen == {"p": False}
    assert vkt.vktGetInt8Matrix() is True
    vkt.vktSetInt8Matrix(False)


def test_stream_is_thread_local(vkt):
    vkt.vktSetStream(0x1234)
    seen = {}

    def other():
        seen["s"] = vkt.vktGetStream()

    th = threading.Thread(target=other)
    th.start()
    th.join()
    assert seen["s"] is None and vkt.vktGetStream() == 0x1234
    vkt.vktSetStream(None)
    assert vkt.vktGetStream() is None


def test_row_pair_threshold_setting(vkt):
    """Per-thread state only: no device work."""
    old = vkt.vktGetRowPairMinCells()
    assert old >= 0
    try:
        vkt.vktSetRowPairMinCells(12345)
        assert vkt.vktGetRowPairMinCells() == 12345
        with pytest.raises(vkt.VktError) as e:
            vkt.vktSetRowPairMinCells(-1)
        assert e.value.code == vkt.vktInvalidValue
        assert vkt.lib().vktGetRowPairMinCells(None) == vkt.vktInvalidValue
    finally:
        vkt.vktSetRowPairMinCells(old)
