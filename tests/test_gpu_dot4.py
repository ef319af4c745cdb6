"""GPU parity of the 8-bit dot-product path: uint8 volumes, integer filters
with k in {3, 5, 7}, weights all in [0, 255] or all in [-128, 127],
sum |w| <= 2048, divisor <= 2^19, rows a multiple of 4 cells.  Results are
integer quotients and must equal the oracle bit for bit.

Shapes put X past one 256-cell tile with a ragged tail (the right x face
inside a tile), at exactly one tile, and at the 4-cell minimum, so every
face-dword case of the staging is exercised; Y and Z are ragged against the
tile rows and slab depths.  The opt-in int8 matrix-core path, which would
take the k = 3 cases with weights in [-128, 127], is kept off here."""
import numpy as np
import pytest

from _gpu import check_against_oracle, run_filter

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def dot_products_only():
    from paper_2203_10213_amd import vkt
    prev = vkt.vktGetInt8Matrix()
    vkt.vktSetInt8Matrix(False)
    yield
    vkt.vktSetInt8Matrix(prev)


MODES = ["clamp", "wrap", "mirror", "border"]
SHAPES = [(1, 1, 4), (3, 2, 8), (5, 1, 72), (9, 33, 64), (20, 40, 260), (7, 19, 256),
          (17, 9, 516), (2, 5, 100)]


def _weights(g, k, signed, budget=2048):
    """Random integer weights in the path's range with sum |w| <= budget."""
    lo, hi = (-128, 127) if signed else (0, 255)
    w = g.integers(lo, hi + 1, (k, k, k)).astype(np.int64)
    s = np.abs(w).sum()
    if s > budget:
        w = np.trunc(w * (budget / s)).astype(np.int64)
    if signed and w.min() >= 0:
        w.flat[0] = -1
    return w.astype(np.int32)


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("k", [3, 5, 7])
@pytest.mark.parametrize("signed", [False, True])
def test_dot4_sweep(orc, mode, k, signed):
    g = np.random.default_rng(700 + 10 * k + MODES.index(mode) + (50 if signed else 0))
    for i, shape in enumerate(SHAPES):
        src = g.integers(0, 256, shape).astype(np.uint8)
        w = _weights(g, k, signed)
        D = [1, 2, 27, 255, 1000, 1 << 19, 64, 7][i]
        out = run_filter(src, w, mode, divisor=D)
        check_against_oracle(orc, src, w, mode, out, divisor=D,
                             what=f"{shape} k={k} signed={signed} D={D}")


@pytest.mark.parametrize("signed", [False, True])
def test_dot4_epilogue_extremes(orc, signed):
    """Largest eligible sums and divisor: every quotient floor((2T+D)/2D)
    must still be exact through the FP32 epilogue; saturation at both ends."""
    g = np.random.default_rng(77 + signed)
    src = g.integers(0, 256, (6, 20, 68)).astype(np.uint8)
    src[:, :, :8] = 255
    src[:, :, 8:16] = 0
    w = np.full((3, 3, 3), -75 if signed else 75, np.int32)  # sum |w| = 2025
    for D in [1, 3, 27, 2025, 2026, 4049, 4050, (1 << 19) - 1, 1 << 19]:
        out = run_filter(src, w, "clamp", divisor=D)
        check_against_oracle(orc, src, w, "clamp", out, divisor=D, what=f"D={D}")


def test_dot4_ties_every_residue(orc):
    """A ramp volume makes T take every residue modulo D, so the half-up
    rule is hit exactly at ties (2T + D divisible by 2D) for even D."""
    x = np.arange(256, dtype=np.int64)
    src = np.broadcast_to((x % 256).astype(np.uint8), (5, 7, 256)).copy()
    src[2] = np.flip(src[2], axis=1)
    w = np.zeros((3, 3, 3), np.int32)
    w[1, 1, 1] = 1
    w[1, 1, 2] = 1  # T = s(x) + s(x+1): all values 0..510
    for D in [2, 4, 6, 10, 16, 50, 100, 510]:
        out = run_filter(src, w, "wrap", divisor=D)
        check_against_oracle(orc, src, w, "wrap", out, divisor=D, what=f"D={D}")


def test_dot4_ineligible_fall_back_exact(orc):
    """Just outside the path's limits (sum |w| > 2048, weights > 255, rows
    not a multiple of 4) the vector FP32/int path runs; still bit-exact."""
    g = np.random.default_rng(78)
    cases = [((4, 9, 64), np.full((3, 3, 3), 80, np.int32), 27),        # sum 2160
             ((4, 9, 64), g.integers(0, 300, (3, 3, 3)).astype(np.int32), 999),
             ((4, 9, 66), np.ones((3, 3, 3), np.int32), 27),
             ((4, 9, 64), np.ones((3, 3, 3), np.int32), (1 << 19) + 1)]
    for shape, w, D in cases:
        src = g.integers(0, 256, shape).astype(np.uint8)
        out = run_filter(src, w, "mirror", divisor=D)
        check_against_oracle(orc, src, w, "mirror", out, divisor=D, what=f"{shape} D={D}")


def test_dot4_box27_phantom_slab(orc):
    """The 512^3 CT-phantom workload's filter (3^3 box, divisor 27) on a
    48-plane slab of the same phantom recipe."""
    from paper_2203_10213_amd import synth
    full = synth.ct_phantom_u8(512, synth.SEEDS["c2a"])
    src = np.ascontiguousarray(full[200:248])
    w = np.ones((3, 3, 3), np.int32)
    out = run_filter(src, w, "clamp", divisor=27)
    check_against_oracle(orc, src, w, "clamp", out, divisor=27, what="phantom slab")
