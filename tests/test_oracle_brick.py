"""Pins of the oracle's BrickDecompose (paper Sec. 3.2, domain decomposition:
bricks of a volume, optionally with ghost cells) against independent
definitions: without ghosts the bricks tile the volume (numpy slicing puts
it back together), with ghosts each brick is a window of numpy's padded
volume, and an interior filtered inside its ghost-extended brick equals
the whole-volume filter there (the property that lets bricks feed the
batched filter)."""
import numpy as np
import pytest

import oracle

MODES = ["clamp", "wrap", "mirror", "border"]
NP_PAD = {"clamp": "edge", "wrap": "wrap", "mirror": "symmetric", "border": "constant"}


def _vol(g, shape, dtype):
    if dtype == np.float32:
        return g.standard_normal(shape).astype(np.float32)
    return g.integers(0, np.iinfo(dtype).max + 1, shape).astype(dtype)


@pytest.mark.parametrize("dtype", [np.uint8, np.uint16, np.float32])
def test_no_ghosts_tiles_the_volume(dtype):
    g = np.random.default_rng(801)
    src = _vol(g, (7, 10, 13), dtype)
    brick = (4, 3, 5)                               # x, y, z
    bricks = oracle.brick_decompose(src, brick)
    assert oracle.brick_grid((13, 10, 7), brick) == (4, 4, 2)
    assert len(bricks) == 4 * 4 * 2
    back = np.zeros_like(src)
    seen = np.zeros(src.shape, int)
    i = 0
    for bz in range(2):
        for by in range(4):
            for bx in range(4):
                b = bricks[i]
                i += 1
                z0, y0, x0 = bz * 5, by * 3, bx * 4
                assert b.shape == (min(5, 7 - z0), min(3, 10 - y0), min(4, 13 - x0))
                back[z0:z0 + b.shape[0], y0:y0 + b.shape[1], x0:x0 + b.shape[2]] = b
                seen[z0:z0 + b.shape[0], y0:y0 + b.shape[1], x0:x0 + b.shape[2]] += 1
    assert (seen == 1).all()
    assert np.array_equal(back, src)


@pytest.mark.parametrize("mode", MODES)
def test_ghosts_are_windows_of_the_padded_volume(mode):
    g = np.random.default_rng(810 + MODES.index(mode))
    for shape, brick, ghost in [((6, 9, 11), (4, 4, 3), (1, 2, 1)),
                                ((5, 5, 5), (2, 2, 2), (3, 3, 3)),     # ghosts wider than bricks
                                ((3, 4, 2), (8, 8, 8), (2, 1, 4)),     # one brick, ghosts > dims
                                ((8, 2, 16), (16, 1, 3), (0, 5, 2))]:
        src = g.random(shape)
        (BX, BY, BZ), (gx, gy, gz) = brick, ghost
        P = np.pad(src, ((gz, gz), (gy, gy), (gx, gx)), mode=NP_PAD[mode])
        Z, Y, X = shape
        nbx, nby, nbz = oracle.brick_grid((X, Y, Z), brick)
        bricks = oracle.brick_decompose(src, brick, ghost, mode)
        i = 0
        for bz in range(nbz):
            for by in range(nby):
                for bx in range(nbx):
                    iz, iy, ix = min(BZ, Z - bz * BZ), min(BY, Y - by * BY), min(BX, X - bx * BX)
                    want = P[bz * BZ:bz * BZ + iz + 2 * gz, by * BY:by * BY + iy + 2 * gy,
                             bx * BX:bx * BX + ix + 2 * gx]
                    assert np.array_equal(bricks[i], want), (mode, shape, brick, ghost, i)
                    i += 1


@pytest.mark.parametrize("mode", MODES)
def test_filtered_brick_interiors_equal_the_whole_volume_filter(mode):
    g = np.random.default_rng(820 + MODES.index(mode))
    src = g.random((9, 12, 14))
    w = g.standard_normal((5, 5, 5))
    r = 2
    T, _ = oracle.correlate(src, w, mode)
    brick = (5, 4, 4)
    nbx, nby, nbz = oracle.brick_grid((14, 12, 9), brick)
    bricks = oracle.brick_decompose(src, brick, (r, r, r), mode)
    i = 0
    for bz in range(nbz):
        for by in range(nby):
            for bx in range(nbx):
                b = bricks[i]
                i += 1
                # the brick's own address mode never reaches its interior
                Tb, _ = oracle.correlate(b, w, "border")
                inner = Tb[r:-r, r:-r, r:-r]
                z0, y0, x0 = bz * 4, by * 4, bx * 5
                want = T[z0:z0 + inner.shape[0], y0:y0 + inner.shape[1], x0:x0 + inner.shape[2]]
                assert np.allclose(inner, want, rtol=0, atol=1e-12)


def test_bad_arguments():
    src = np.zeros((2, 2, 2), np.uint8)
    with pytest.raises(Exception):
        oracle.brick_decompose(src, (1, 1, 1), (0, 0, 0), 7)
