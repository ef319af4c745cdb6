"""GPU parity of vktApplyFilterRange: inside the half-open region the output
equals the oracle's whole-volume result (same tolerances as ApplyFilter:
the source is addressed through the whole volume and the address mode);
every cell outside the region keeps its previous contents (a sentinel)."""
import numpy as np
import pytest

from _gpu import check_against_oracle, run_filter

pytestmark = pytest.mark.gpu

SENTINEL = {np.dtype(np.float32): np.float32(np.nan), np.dtype(np.uint8): np.uint8(0xA5),
            np.dtype(np.uint16): np.uint16(0xA5A5)}


def _outside_untouched(out, roi, what):
    (x0, y0, z0), (x1, y1, z1) = roi
    inside = np.zeros(out.shape, bool)
    inside[z0:z1, y0:y1, x0:x1] = True
    sent = np.full(out.shape, SENTINEL[out.dtype], out.dtype)
    same = (out.view(np.uint8).reshape(*out.shape, -1) ==
            sent.view(np.uint8).reshape(*out.shape, -1)).all(axis=-1)
    bad = np.argwhere(~inside & ~same)
    assert bad.size == 0, f"{what}: {len(bad)} cells outside the region changed, first {bad[:3].tolist()}"


def _rois(g, shape, n):
    """Random regions plus the edge cases: whole volume, one cell, faces."""
    Z, Y, X = shape
    out = [((0, 0, 0), (X, Y, Z)), ((X - 1, Y - 1, Z - 1), (X, Y, Z)),
           ((0, 0, 0), (1, 1, 1)), ((1, 0, Z // 2), (X, Y - 1, Z))]
    for _ in range(n):
        lo = [int(g.integers(0, d)) for d in (X, Y, Z)]
        hi = [int(g.integers(l + 1, d + 1)) for l, d in zip(lo, (X, Y, Z))]
        out.append((tuple(lo), tuple(hi)))
    return out


CASES = [
    # (dtype, shape (Z, Y, X), k, weight kind, precision)  -> path exercised
    (np.float32, (9, 40, 70), 3, "float", "fp32"),          # VALU FP32
    (np.uint16, (7, 35, 66), 5, "float", "fp32"),           # VALU FP32, integer cells
    (np.uint8, (8, 33, 264), 3, "int_u", "auto"),           # dot4 when the region is 4-aligned
    (np.uint8, (6, 20, 67), 5, "int_s", "auto"),            # VALU exact integer (odd rows)
    (np.float32, (12, 70, 40), 7, "float", "auto"),         # MFMA 16x16 bf16 x6
    (np.uint16, (20, 33, 37), 9, "float", "auto"),          # MFMA 32x32 fp16
    (np.float32, (10, 131, 70), 7, "float", "splitbf16"),   # MFMA 16x16 bf16 x3
    (np.uint8, (9, 70, 45), 5, "float", "auto"),            # MFMA 16x16 fp16, k = 5
    (np.uint16, (8, 67, 99), 7, "float", "auto"),           # MFMA 16x16 fp16 x4
    # the row-pair kernel, forced for these small regions (threshold 0):
    (np.float32, (10, 131, 70), 7, "float", "splitbf16", "rp"),  # bf16 x3, 3 tile rows
    (np.uint8, (9, 70, 45), 5, "float", "auto", "rp"),           # fp16, k = 5
    (np.float32, (11, 66, 37), 5, "float", "auto", "rp"),        # bf16 x6, k = 5
]


@pytest.mark.parametrize("mode", ["clamp", "mirror", "border", "wrap"])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_range_matches_oracle_inside_and_keeps_outside(orc, mode, case):
    from paper_2203_10213_amd import vkt
    dtype, shape, k, kind, precision = CASES[case][:5]
    rp = vkt.vktGetRowPairMinCells()
    if CASES[case][5:] == ("rp",):
        vkt.vktSetRowPairMinCells(0)
    try:
        _range_case(orc, mode, case, dtype, shape, k, kind, precision)
    finally:
        vkt.vktSetRowPairMinCells(rp)


def _range_case(orc, mode, case, dtype, shape, k, kind, precision):
    g = np.random.default_rng(900 + 7 * case + len(mode))
    if dtype == np.float32:
        src = g.standard_normal(shape).astype(np.float32)
    else:
        src = g.integers(0, np.iinfo(dtype).max + 1, shape).astype(dtype)
    D = None
    if kind == "float":
        w = g.standard_normal((k, k, k)).astype(np.float32)
        if dtype != np.float32:
            w = (np.abs(w) / np.abs(w).sum()).astype(np.float32)
    elif kind == "int_u":
        w, D = g.integers(0, 4, (k, k, k)).astype(np.int32), 27
    else:
        w, D = g.integers(-3, 4, (k, k, k)).astype(np.int32), 5
    rois = _rois(g, shape, 4)
    if kind == "int_u":  # 4-aligned x bounds run the dot-product path
        rois.append(((4, 1, 1), (260, shape[1] - 2, shape[0] - 1)))
    for roi in rois:
        out = run_filter(src, w, mode, divisor=D, precision=precision, roi=roi)
        what = f"{dtype.__name__} k={k} {mode} roi={roi}"
        check_against_oracle(orc, src, w, mode, out, divisor=D, roi=roi, what=what)
        _outside_untouched(out, roi, what)


def test_range_empty_and_invalid():
    import torch
    from paper_2203_10213_amd import vkt
    from _gpu import sentinel_like, to_device
    src = to_device(np.ones((4, 5, 6), np.float32))
    dst = sentinel_like(src)
    hs, hd = vkt.volume_from_tensor(src), vkt.volume_from_tensor(dst)
    hf = vkt.vktFilterCreate(np.ones((3, 3, 3), np.float32) / 27)
    try:
        vkt.vktSetStream(torch.cuda.current_stream())
        vkt.vktApplyFilterRange(hd, hs, hf, (2, 2, 2), (2, 5, 4))  # empty: no-op
        for first, last in [((3, 0, 0), (2, 5, 4)), ((0, 0, 0), (7, 5, 4)),
                            ((-1, 0, 0), (6, 5, 4)), ((0, 0, 0), (6, 6, 4))]:
            with pytest.raises(vkt.VktError) as e:
                vkt.vktApplyFilterRange(hd, hs, hf, first, last)
            assert e.value.code == vkt.vktInvalidValue
        vkt.vktSynchronize()
        assert torch.isnan(dst).all()  # nothing was written
    finally:
        vkt.vktFilterDestroy(hf)
        vkt.vktStructuredVolumeDestroy(hs)
        vkt.vktStructuredVolumeDestroy(hd)
