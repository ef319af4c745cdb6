"""GPU parity of the int8 matrix-core path: uint8 volumes, 3x3x3 integer
filters with weights in [-128, 127], sum |w| <= 2048, divisor <= 2^19, rows
a multiple of 4 cells.  Results are integer quotients and must equal the
oracle bit for bit, and equal the 8-bit dot-product path's.

The tile is 64 x 64 cells and each wave splits its 64 columns into four
16-cell x-tiles whose edge cells come from a separate staged entry, so the
shapes put the right x face inside a 16-cell x-tile (X - x0 not a multiple
of 16), exactly on an x-tile boundary (the face cell is an edge cell), on a
64-cell tile boundary, and at the 4-cell minimum; Y and Z are ragged against
the 16-row bands, the 64-row tiles and the slab depths."""
import numpy as np
import pytest

from _gpu import check_against_oracle, run_filter, sample_points, to_device

pytestmark = pytest.mark.gpu

MODES = ["clamp", "wrap", "mirror", "border"]
SHAPES = [(1, 1, 4), (3, 2, 8), (5, 1, 72), (9, 33, 64), (4, 65, 80), (7, 19, 128),
          (11, 70, 132), (2, 5, 100), (13, 17, 196), (6, 130, 36)]


def _weights(g, budget=2048):
    w = g.integers(-128, 128, (3, 3, 3)).astype(np.int64)
    s = np.abs(w).sum()
    if s > budget:
        w = np.trunc(w * (budget / s)).astype(np.int64)
    return w.astype(np.int32)


@pytest.fixture
def int8_matrix():
    from paper_2203_10213_amd import vkt
    prev = vkt.vktGetInt8Matrix()
    vkt.vktSetInt8Matrix(True)
    yield vkt
    vkt.vktSetInt8Matrix(prev)


@pytest.mark.parametrize("mode", MODES)
def test_i8mma_sweep(orc, int8_matrix, mode):
    g = np.random.default_rng(900 + MODES.index(mode))
    Ds = [1, 2, 27, 255, 1000, 1 << 19, 64, 7, 3, 100]
    for i, shape in enumerate(SHAPES):
        src = g.integers(0, 256, shape).astype(np.uint8)
        w = _weights(g)
        out = run_filter(src, w, mode, divisor=Ds[i])
        check_against_oracle(orc, src, w, mode, out, divisor=Ds[i],
                             what=f"{shape} D={Ds[i]}")


def test_i8mma_matches_dot_products(int8_matrix):
    """The same calls with the matrix path off (8-bit dot products): the
    stored volumes are identical."""
    vkt = int8_matrix
    g = np.random.default_rng(910)
    for shape, mode in [((21, 70, 196), "clamp"), ((9, 64, 256), "mirror"),
                        ((5, 33, 68), "wrap"), ((8, 40, 144), "border")]:
        src = g.integers(0, 256, shape).astype(np.uint8)
        w = _weights(g)
        D = int(np.abs(w).sum()) or 1
        vkt.vktSetInt8Matrix(True)
        a = run_filter(src, w, mode, divisor=D)
        vkt.vktSetInt8Matrix(False)
        b = run_filter(src, w, mode, divisor=D)
        assert np.array_equal(a, b), f"{shape} {mode}"


def test_i8mma_epilogue_extremes(orc, int8_matrix):
    """Largest eligible sums and divisor, both signs: every quotient
    floor((2T+D)/2D) exact through the FP32 epilogue; saturation at both
    ends."""
    g = np.random.default_rng(920)
    src = g.integers(0, 256, (6, 20, 68)).astype(np.uint8)
    src[:, :, :8] = 255
    src[:, :, 8:16] = 0
    for wv in (-75, 75):
        w = np.full((3, 3, 3), wv, np.int32)  # sum |w| = 2025
        for D in [1, 3, 27, 2025, 2026, 4049, 4050, (1 << 19) - 1, 1 << 19]:
            out = run_filter(src, w, "clamp", divisor=D)
            check_against_oracle(orc, src, w, "clamp", out, divisor=D, what=f"w={wv} D={D}")


def test_i8mma_single_taps(orc, int8_matrix):
    """One nonzero weight at each of the 27 positions (weight -128 or 127):
    every tap's placement in the Toeplitz operand, the edge cells included,
    is checked on its own."""
    g = np.random.default_rng(930)
    src = g.integers(0, 256, (5, 37, 72)).astype(np.uint8)
    for pos in range(27):
        w = np.zeros(27, np.int32)
        w[pos] = -128 if pos % 2 else 127
        w = w.reshape(3, 3, 3)
        out = run_filter(src, w, "mirror", divisor=2 + pos)
        check_against_oracle(orc, src, w, "mirror", out, divisor=2 + pos, what=f"tap {pos}")


def test_i8mma_ranges(orc, int8_matrix):
    """ApplyFilterRange on the matrix path: x bounds multiples of 4 (tiles
    start at the range's x0), cells outside the range untouched."""
    g = np.random.default_rng(940)
    src = g.integers(0, 256, (12, 50, 136)).astype(np.uint8)
    w = _weights(g)
    for roi in [((4, 3, 2), (132, 47, 11)), ((0, 0, 0), (136, 50, 12)),
                ((68, 17, 5), (72, 18, 6)), ((12, 1, 0), (80, 49, 3))]:
        out = run_filter(src, w, "wrap", divisor=97, roi=roi)
        check_against_oracle(orc, src, w, "wrap", out, divisor=97, roi=roi, what=str(roi))
        (x0, y0, z0), (x1, y1, z1) = roi
        mask = np.ones(src.shape, bool)
        mask[z0:z1, y0:y1, x0:x1] = False
        assert (out[mask] == 0xA5).all(), f"{roi}: cells outside the range written"


def test_i8mma_full_size_phantom_matches_dot_products(orc, int8_matrix):
    """The 512^3 CT-phantom workload (3^3 box / 27) and a signed 3^3 filter:
    the matrix path equals the dot-product path on every cell, and the
    oracle on sampled cells."""
    import torch
    from paper_2203_10213_amd import synth
    vkt = int8_matrix
    src = synth.ct_phantom_u8(512, synth.SEEDS["c2a"])
    s = to_device(src)
    g = np.random.default_rng(950)
    for w, D in [(np.ones((3, 3, 3), np.int32), 27), (_weights(g), 613)]:
        vkt.vktSetInt8Matrix(True)
        a = run_filter(src, w, "clamp", divisor=D, src_t=s)
        vkt.vktSetInt8Matrix(False)
        b = run_filter(src, w, "clamp", divisor=D, src_t=s)
        assert np.array_equal(a, b)
        pts = sample_points(src.shape, 3000, 951)
        check_against_oracle(orc, src, w, "clamp", a, divisor=D, pts=pts, what=f"D={D}")
        del a, b
    del s
    torch.cuda.empty_cache()
