"""vktGetFilterPath reports the path the planner takes for a call (the same
planning code as vktApplyFilter), with the number of split products."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _reset():
    from paper_2203_10213_amd import vkt
    yield
    vkt.vktSetPrecision("auto")
    vkt.vktSetSeparable(False)
    vkt.vktSetInt8Matrix(False)


def _path(vkt, shape, dtype, w, divisor=None):
    import torch
    src = torch.zeros(shape, dtype=dtype, device="cuda")
    dst = torch.zeros_like(src)
    hs, hd = vkt.volume_from_tensor(src), vkt.volume_from_tensor(dst)
    hf = vkt.vktFilterCreate(w) if divisor is None else vkt.vktFilterCreateInt(w, divisor)
    try:
        return vkt.vktGetFilterPath(hd, hs, hf, "clamp")
    finally:
        vkt.vktFilterDestroy(hf)
        vkt.vktStructuredVolumeDestroy(hs)
        vkt.vktStructuredVolumeDestroy(hd)


def test_paths_and_products():
    import torch
    from paper_2203_10213_amd import synth, vkt
    g7 = synth.random_l1(7, 1)
    box, D = synth.box_int(3)
    f32, u8, u16 = torch.float32, torch.uint8, torch.uint16
    vkt.vktSetPrecision("splitbf16")
    assert _path(vkt, (8, 8, 8), f32, g7) == (vkt.vktFilterPathSplitMatrix, 3)
    assert _path(vkt, (8, 8, 8), u8, np.abs(g7)) == (vkt.vktFilterPathSplitMatrix, 2)
    assert _path(vkt, (8, 8, 8), u16, np.abs(g7)) == (vkt.vktFilterPathSplitMatrix, 4)
    vkt.vktSetPrecision("splitbf16x6")
    assert _path(vkt, (8, 8, 8), f32, g7) == (vkt.vktFilterPathSplitMatrix, 6)
    vkt.vktSetPrecision("fp32")
    assert _path(vkt, (8, 8, 8), f32, g7) == (vkt.vktFilterPathVectorFP32, 1)
    # k < 5 stays on the vector ALUs in every precision
    vkt.vktSetPrecision("auto")
    assert _path(vkt, (8, 8, 8), f32, synth.gaussian_weights(3, 1.0))[0] == \
        vkt.vktFilterPathVectorFP32
    # uint8 box/27: 8-bit dot products (rows of a multiple of 4 cells), else
    # the exact vector path; int8 matrix cores when enabled
    assert _path(vkt, (8, 8, 8), u8, box, D) == (vkt.vktFilterPathDot8, 1)
    assert _path(vkt, (8, 8, 7), u8, box, D) == (vkt.vktFilterPathVectorFP32, 1)
    vkt.vktSetInt8Matrix(True)
    assert _path(vkt, (8, 8, 8), u8, box, D) == (vkt.vktFilterPathInt8Matrix, 1)
    vkt.vktSetInt8Matrix(False)
    # rank-1 form when enabled (a 5^3 Gaussian is separable)
    vkt.vktSetSeparable(True)
    assert _path(vkt, (8, 8, 8), f32, synth.gaussian_weights(5, 1.5)) == \
        (vkt.vktFilterPathSeparable, 1)
    assert _path(vkt, (8, 8, 8), f32, g7)[0] == vkt.vktFilterPathSplitMatrix


def test_path_errors():
    import torch
    from paper_2203_10213_amd import vkt
    a = torch.zeros((4, 4, 4), dtype=torch.float32, device="cuda")
    ha = vkt.volume_from_tensor(a)
    hf = vkt.vktFilterCreate(np.ones((3, 3, 3), np.float32))
    try:
        with pytest.raises(vkt.VktError):   # dst == src
            vkt.vktGetFilterPath(ha, ha, hf)
        assert vkt.lib().vktGetFilterPath(ha, ha, hf, 0, None, None) == vkt.vktInvalidValue
    finally:
        vkt.vktFilterDestroy(hf)
        vkt.vktStructuredVolumeDestroy(ha)
