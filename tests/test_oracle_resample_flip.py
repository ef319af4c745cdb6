"""Pins of the oracle's Resample and Flip (paper Sec. 3.2; the structured
benchmarks of Sec. 4 downscale by two and flip along the longest axis)
against independent definitions: block means, scipy's linear interpolation
at the mapped cell centres, exact reproduction of linear functions, and
numpy's flip."""
import numpy as np
import pytest

import oracle


def _vol(g, shape, dtype):
    if dtype == np.float32:
        return g.standard_normal(shape).astype(np.float32)
    return g.integers(0, np.iinfo(dtype).max + 1, shape).astype(dtype)


@pytest.mark.parametrize("dtype", [np.uint8, np.uint16, np.float32])
def test_half_downscale_is_block_mean(dtype):
    g = np.random.default_rng(31)
    src = _vol(g, (6, 10, 14), dtype)
    out, A = oracle.resample(src, (7, 5, 3))
    want = src.astype(np.float64).reshape(3, 2, 5, 2, 7, 2).mean(axis=(1, 3, 5))
    assert np.allclose(out, want, rtol=0, atol=1e-12 * max(1.0, np.abs(want).max()))
    if dtype != np.float32:
        assert np.array_equal(out, A)  # non-negative cells: sum |w s| = sum w s


def test_same_size_is_copy():
    g = np.random.default_rng(32)
    src = _vol(g, (5, 7, 9), np.float32)
    out, _ = oracle.resample(src, (9, 7, 5))
    assert np.array_equal(out, src.astype(np.float64))


@pytest.mark.parametrize("dims", [(13, 5, 4), (20, 11, 7), (3, 17, 9), (1, 1, 1)])
def test_matches_scipy_linear_at_mapped_centres(dims):
    from scipy import ndimage
    g = np.random.default_rng(33)
    src = g.standard_normal((6, 9, 11))
    Xo, Yo, Zo = dims
    out, _ = oracle.resample(src, dims)
    Z, Y, X = src.shape
    cz = (np.arange(Zo) + 0.5) * Z / Zo - 0.5
    cy = (np.arange(Yo) + 0.5) * Y / Yo - 0.5
    cx = (np.arange(Xo) + 0.5) * X / Xo - 0.5
    zz, yy, xx = np.meshgrid(cz, cy, cx, indexing="ij")
    want = ndimage.map_coordinates(src, [zz, yy, xx], order=1, mode="nearest")
    assert np.allclose(out, want, rtol=0, atol=1e-12)


def test_linear_function_reproduced_inside():
    # f = 3x - 2y + 0.5z + 7 on the source grid; every destination centre that
    # maps inside [0, n-1] on all axes gets f at the mapped position exactly
    Z, Y, X = 7, 8, 9
    z, y, x = np.meshgrid(np.arange(Z), np.arange(Y), np.arange(X), indexing="ij")
    src = (3.0 * x - 2.0 * y + 0.5 * z + 7.0)
    Xo, Yo, Zo = 17, 5, 12
    out, _ = oracle.resample(src, (Xo, Yo, Zo))
    ux = (np.arange(Xo) + 0.5) * X / Xo - 0.5
    uy = (np.arange(Yo) + 0.5) * Y / Yo - 0.5
    uz = (np.arange(Zo) + 0.5) * Z / Zo - 0.5
    UZ, UY, UX = np.meshgrid(uz, uy, ux, indexing="ij")
    inside = (UX >= 0) & (UX <= X - 1) & (UY >= 0) & (UY <= Y - 1) & (UZ >= 0) & (UZ <= Z - 1)
    want = 3.0 * UX - 2.0 * UY + 0.5 * UZ + 7.0
    assert inside.sum() > 100
    assert np.allclose(out[inside], want[inside], rtol=0, atol=1e-12)


@pytest.mark.parametrize("dtype", [np.uint8, np.uint16, np.float32])
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_flip_is_numpy_flip_and_an_involution(dtype, axis):
    g = np.random.default_rng(34 + axis)
    src = _vol(g, (4, 6, 5), dtype)
    out = oracle.flip(src, axis)
    assert np.array_equal(out, np.flip(src, axis=2 - axis))
    assert np.array_equal(oracle.flip(out, axis), src)


def test_bad_arguments():
    with pytest.raises(Exception):
        oracle.flip(np.zeros((2, 2, 2), np.float32), 3)
    with pytest.raises(Exception):
        oracle.resample(np.zeros((2, 2, 2), np.float32), (0, 1, 1))
