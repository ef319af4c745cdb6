"""Pins that tie the FP64 oracle to the paper and to mathematics, not to itself.

Paper: volkit, Sec. 3.2 "Volume Manipulation": ApplyFilter applies a user
convolution kernel (edge detection, Gaussian blur) and can be written with
Transform, one computation per cell; Fig. 4 gives the Fill/FillRange example.
Each test below fixes the oracle against something independent of its code:
hand-typed tables, a library routine that reduces to the same operation,
closed forms, invariants, or a brute force written differently.
"""
import itertools
import json
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.ndimage as ndi

GOLD = os.path.join(os.path.dirname(__file__), "golden")
MODES = ["clamp", "wrap", "mirror", "border"]
SCIPY_MODE = {"clamp": "nearest", "wrap": "wrap", "mirror": "reflect",
              "border": "constant"}
NP_PAD = {"clamp": "edge", "wrap": "wrap", "mirror": "symmetric",
          "border": "constant"}


# ------------------------------------------------------------ address map --

def test_address_tables(orc):
    """Hand-typed extension of a 3-cell axis [a b c] for i = -7..8."""
    i = list(range(-7, 9))
    want = {
        "clamp":  [0, 0, 0, 0, 0, 0, 0, 0, 1, 2, 2, 2, 2, 2, 2, 2],
        "wrap":   [2, 0, 1, 2, 0, 1, 2, 0, 1, 2, 0, 1, 2, 0, 1, 2],
        # ... c b a | a b c | c b a | a b c ...  (edge cell repeated)
        "mirror": [0, 0, 1, 2, 2, 1, 0, 0, 1, 2, 2, 1, 0, 0, 1, 2],
        "border": [-1] * 7 + [0, 1, 2] + [-1] * 6,
    }
    for m, exp in want.items():
        assert [orc.address(v, 3, m) for v in i] == exp, m
    assert [orc.address(v, 1, "mirror") for v in (-3, -1, 0, 1, 4)] == [0] * 5
    assert [orc.address(v, 1, "wrap") for v in (-3, -1, 0, 1, 4)] == [0] * 5


# ------------------------------------------------- library special cases --

def _rand_case(g, kmax=7, dmax=9):
    dims = tuple(int(v) for v in g.integers(1, dmax + 1, 3))
    k = int(g.choice([v for v in (1, 3, 5, 7, 9) if v <= kmax]))
    return dims, k


@pytest.mark.parametrize("mode", MODES)
def test_matches_scipy_correlate(orc, mode):
    """Random tiny volumes (dims 1..9, including dims below the filter
    radius) and random asymmetric filters: the oracle's T equals
    scipy.ndimage.correlate in FP64 with the matching boundary rule.  An
    asymmetric filter pins the orientation (correlation, no flip) and the
    axis order w[c, b, a]."""
    g = np.random.default_rng(11 + MODES.index(mode))
    for _ in range(60):
        dims, k = _rand_case(g)
        src = g.standard_normal(dims)
        w = g.standard_normal((k, k, k))
        T, A = orc.correlate(src, w, mode)
        ref = ndi.correlate(src, w, mode=SCIPY_MODE[mode], cval=0.0)
        scale = ndi.correlate(np.abs(src), np.abs(w), mode=SCIPY_MODE[mode])
        assert np.allclose(T, ref, rtol=0, atol=1e-12 * max(1.0, scale.max()))
        assert np.allclose(A, scale, rtol=1e-13, atol=1e-300)


@pytest.mark.parametrize("dtype", [np.uint8, np.uint16, np.float32])
def test_formats_widen_exactly(orc, dtype):
    """Stored formats are widened exactly to FP64 before the sum."""
    g = np.random.default_rng(5)
    if dtype == np.float32:
        src = g.standard_normal((6, 7, 8)).astype(dtype)
    else:
        src = g.integers(0, np.iinfo(dtype).max + 1, (6, 7, 8)).astype(dtype)
    w = g.standard_normal((3, 3, 3))
    T, _ = orc.correlate(src, w, "clamp")
    ref = ndi.correlate(src.astype(np.float64), w, mode="nearest")
    assert np.allclose(T, ref, rtol=1e-13, atol=1e-9)


# ----------------------------------------------------------- brute force --

def _brute(src, w, mode):
    """Padding-based brute force: extend the volume by r on each side with
    numpy's pad rule, then add k^3 shifted copies weighted by the taps."""
    k = w.shape[0]
    r = (k - 1) // 2
    P = np.pad(src.astype(np.float64), r, mode=NP_PAD[mode])
    Z, Y, X = src.shape
    out = np.zeros(src.shape, np.float64)
    for c, b, a in itertools.product(range(k), repeat=3):
        out += w[c, b, a] * P[c:c + Z, b:b + Y, a:a + X]
    return out


@pytest.mark.parametrize("mode", MODES)
def test_matches_padding_brute_force(orc, mode):
    g = np.random.default_rng(21 + MODES.index(mode))
    for _ in range(40):
        dims, k = _rand_case(g, kmax=9, dmax=8)
        src = g.random(dims)
        w = g.standard_normal((k, k, k))
        T, _ = orc.correlate(src, w, mode)
        assert np.allclose(T, _brute(src, w, mode), rtol=0, atol=1e-11)


def test_pure_python_loops_tiny(orc):
    """Fully explicit pure-Python loops (no numpy arithmetic) on a 3x2x4
    volume with k = 3 and k = 5 under clamp."""
    g = np.random.default_rng(3)
    src = g.integers(0, 256, (3, 2, 4)).astype(np.uint8)
    for k in (3, 5):
        r = k // 2
        w = g.integers(-4, 5, (k, k, k)).astype(np.float64)
        T, _ = orc.correlate(src, w, "clamp")
        Z, Y, X = src.shape
        for z in range(Z):
            for y in range(Y):
                for x in range(X):
                    t = 0
                    for c in range(k):
                        for b in range(k):
                            for a in range(k):
                                zz = min(max(z + c - r, 0), Z - 1)
                                yy = min(max(y + b - r, 0), Y - 1)
                                xx = min(max(x + a - r, 0), X - 1)
                                t += int(w[c, b, a]) * int(src[zz, yy, xx])
                    assert T[z, y, x] == t


# ------------------------------------------------------ invariants, pins --

@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("dtype", [np.uint8, np.uint16, np.float32])
def test_centred_delta_is_identity(orc, mode, dtype):
    g = np.random.default_rng(7)
    if dtype == np.float32:
        src = g.standard_normal((5, 6, 9)).astype(dtype)
    else:
        src = g.integers(0, np.iinfo(dtype).max + 1, (5, 6, 9)).astype(dtype)
    for k in (1, 3, 7):
        w = np.zeros((k, k, k), np.float32)
        w[k // 2, k // 2, k // 2] = 1.0
        out = orc.apply_filter(src, w, mode)
        assert out.dtype == src.dtype and np.array_equal(out, src)
        wi = np.zeros((k, k, k), np.int32)
        wi[k // 2, k // 2, k // 2] = 3
        out = orc.apply_filter(src, wi, mode, divisor=3)
        if dtype == np.float32:
            assert np.array_equal(out, src)
        else:
            assert np.array_equal(out, src)


def test_off_centre_delta_orientation_and_modes(orc):
    """1-D worked example on a 5-cell row [10 20 30 40 50] (Y = Z = 1) with
    a 3-tap delta at a = 2 (reads x + 1) and at a = 0 (reads x - 1)."""
    src = np.array([10, 20, 30, 40, 50], np.float32).reshape(1, 1, 5)
    plus = {"clamp": [20, 30, 40, 50, 50], "wrap": [20, 30, 40, 50, 10],
            "mirror": [20, 30, 40, 50, 50], "border": [20, 30, 40, 50, 0]}
    minus = {"clamp": [10, 10, 20, 30, 40], "wrap": [50, 10, 20, 30, 40],
             "mirror": [10, 10, 20, 30, 40], "border": [0, 10, 20, 30, 40]}
    for a, table in ((2, plus), (0, minus)):
        w = np.zeros((3, 3, 3))
        w[1, 1, a] = 1.0
        for m in MODES:
            T, _ = orc.correlate(src, w, m)
            assert T.ravel().tolist() == table[m], (a, m)
    # the same along y and z: tap b = 2 reads y + 1, tap c = 2 reads z + 1
    vol = np.arange(2 * 3 * 4, dtype=np.float64).reshape(2, 3, 4)
    w = np.zeros((3, 3, 3))
    w[1, 2, 1] = 1.0
    T, _ = orc.correlate(vol, w, "clamp")
    assert np.array_equal(T[:, :2, :], vol[:, 1:, :])
    assert np.array_equal(T[:, 2, :], vol[:, 2, :])
    w = np.zeros((3, 3, 3))
    w[2, 1, 1] = 1.0
    T, _ = orc.correlate(vol, w, "clamp")
    assert np.array_equal(T[0], vol[1]) and np.array_equal(T[1], vol[1])


@pytest.mark.parametrize("mode", ["clamp", "wrap", "mirror"])
def test_constant_volume_normalised_filter(orc, mode):
    """A normalised filter keeps a constant volume: float weights give
    c * sum(w_fp32); the integer box / k^3 gives exactly c."""
    from paper_2203_10213_amd import synth
    for k in (3, 5, 7):
        w = synth.gaussian_weights(k, 1.3)
        src = np.full((4, 5, 6), 0.7, np.float32)
        T, _ = orc.correlate(src, w, mode)
        want = float(np.float32(0.7)) * float(w.astype(np.float64).sum())
        assert np.allclose(T, want, rtol=1e-15, atol=0)
        wi, D = synth.box_int(k)
        for val in (0, 1, 77, 255):
            s8 = np.full((3, 4, 5), val, np.uint8)
            assert np.all(orc.apply_filter(s8, wi, mode, divisor=D) == val)


def test_border_constant_volume_loses_mass(orc):
    """Zero border: an all-ones volume under the box sum counts the
    in-volume neighbours, a closed form per cell."""
    src = np.ones((3, 4, 5))
    T, _ = orc.correlate(src, np.ones((3, 3, 3)), "border")
    cnt = [[[len([1 for c in (-1, 0, 1) if 0 <= z + c < 3])
             * len([1 for b in (-1, 0, 1) if 0 <= y + b < 4])
             * len([1 for a in (-1, 0, 1) if 0 <= x + a < 5])
             for x in range(5)] for y in range(4)] for z in range(3)]
    assert np.array_equal(T, np.array(cnt, np.float64))


def test_box_filter_is_neighbourhood_mean(orc):
    """Integer box / 27 on u8 equals the half-up rounded mean of the clamped
    3x3x3 neighbourhood, computed with exact fractions."""
    g = np.random.default_rng(9)
    for dims in [(1, 1, 1), (2, 1, 3), (3, 4, 5), (5, 2, 2)]:
        src = g.integers(0, 256, dims).astype(np.uint8)
        wi, D = np.ones((3, 3, 3), np.int32), 27
        out = orc.apply_filter(src, wi, "clamp", divisor=D)
        Z, Y, X = dims
        for z, y, x in itertools.product(range(Z), range(Y), range(X)):
            s = sum(int(src[min(max(z + c, 0), Z - 1), min(max(y + b, 0), Y - 1),
                            min(max(x + a, 0), X - 1)])
                    for c in (-1, 0, 1) for b in (-1, 0, 1) for a in (-1, 0, 1))
            m = Fraction(s, 27) + Fraction(1, 2)
            assert out[z, y, x] == min(255, m.numerator // m.denominator)


def test_separable_gaussian_equals_three_1d_passes(orc):
    """A separable Gaussian with FP64 weights equals three 1-D passes
    (scipy correlate1d along x, y, z) to ~1e-12."""
    g = np.random.default_rng(4)
    src = g.random((12, 13, 14))
    for k, sigma in ((3, 1.0), (5, 1.5), (7, 2.0), (11, 2.5)):
        r = k // 2
        g1 = np.exp(-np.arange(-r, r + 1) ** 2 / (2 * sigma * sigma))
        g1 /= g1.sum()
        w3 = g1[:, None, None] * g1[None, :, None] * g1[None, None, :]
        for m in MODES:
            T, _ = orc.correlate(src, w3, m)
            sm = SCIPY_MODE[m]
            ref = ndi.correlate1d(src, g1, axis=2, mode=sm)
            ref = ndi.correlate1d(ref, g1, axis=1, mode=sm)
            ref = ndi.correlate1d(ref, g1, axis=0, mode=sm)
            assert np.allclose(T, ref, rtol=0, atol=1e-12), (k, m)


def test_wrap_equals_fft_circular_correlation(orc):
    g = np.random.default_rng(8)
    n = (16, 12, 20)
    src = g.standard_normal(n)
    for k in (3, 5, 7):
        r = k // 2
        w = g.standard_normal((k, k, k))
        h = np.zeros(n)
        for c, b, a in itertools.product(range(k), repeat=3):
            h[(r - c) % n[0], (r - b) % n[1], (r - a) % n[2]] += w[c, b, a]
        ref = np.real(np.fft.ifftn(np.fft.fftn(src) * np.fft.fftn(h)))
        T, _ = orc.correlate(src, w, "wrap")
        assert np.allclose(T, ref, rtol=0, atol=1e-10)
        # exact translation equivariance under wrap
        sh = np.roll(src, (3, -2, 5), axis=(0, 1, 2))
        T2, _ = orc.correlate(sh, w, "wrap")
        assert np.array_equal(T2, np.roll(T, (3, -2, 5), axis=(0, 1, 2))) or \
            np.allclose(T2, np.roll(T, (3, -2, 5), axis=(0, 1, 2)), atol=1e-13)


@pytest.mark.parametrize("mode", MODES)
def test_linearity(orc, mode):
    g = np.random.default_rng(12)
    u, v = g.standard_normal((2, 7, 6, 9))
    w = g.standard_normal((5, 5, 5))
    al, be = 0.75, -1.25
    lhs, _ = orc.correlate(al * u + be * v, w, mode)
    fu, _ = orc.correlate(u, w, mode)
    fv, _ = orc.correlate(v, w, mode)
    assert np.allclose(lhs, al * fu + be * fv, rtol=0, atol=1e-12)


@pytest.mark.parametrize("mode", MODES)
def test_axis_permutation_commutes(orc, mode):
    g = np.random.default_rng(13)
    src = g.standard_normal((5, 7, 9))
    w = g.standard_normal((3, 3, 3))
    T, _ = orc.correlate(src, w, mode)
    for perm in itertools.permutations(range(3)):
        Tp, _ = orc.correlate(np.ascontiguousarray(src.transpose(perm)),
                              np.ascontiguousarray(w.transpose(perm)), mode)
        assert np.allclose(Tp, T.transpose(perm), rtol=0, atol=1e-12)


def test_rounding_golden(orc):
    """Hand-computed stored values (half-up, saturation, exact divisor)."""
    cases = json.load(open(os.path.join(GOLD, "rounding_cases.json")))["cases"]
    dt = {"u8": np.uint8, "u16": np.uint16, "f32": np.float32}
    for fmt, s, w, D, want in cases:
        src = np.array(s, dt[fmt]).reshape(1, 1, 1)
        if D is None:
            out = orc.apply_filter(src, np.array(w, np.float32).reshape(1, 1, 1))
        else:
            out = orc.apply_filter(src, np.array(w, np.int32).reshape(1, 1, 1),
                                   divisor=D)
        assert out.ravel()[0] == want, (fmt, s, w, D)


def test_points_agree_with_full_volume(orc):
    g = np.random.default_rng(14)
    src = g.integers(0, 65536, (9, 10, 11)).astype(np.uint16)
    w = g.standard_normal((5, 5, 5))
    for m in MODES:
        T, A = orc.correlate(src, w, m)
        pts = np.stack([g.integers(0, 11, 50), g.integers(0, 10, 50),
                        g.integers(0, 9, 50)], 1)
        Tp, Ap = orc.correlate_points(src, w, m, pts)
        assert np.array_equal(Tp, T[pts[:, 2], pts[:, 1], pts[:, 0]])
        assert np.array_equal(Ap, A[pts[:, 2], pts[:, 1], pts[:, 0]])


def test_box_agrees_with_full_volume(orc):
    """The box form equals the (pinned) whole-volume sum on its cells, for
    boxes touching every face, interior boxes, empty boxes and any thread
    count; the address mode acts at the volume's faces, not the box's."""
    g = np.random.default_rng(16)
    src = g.integers(0, 256, (11, 9, 13)).astype(np.uint8)
    w = g.standard_normal((5, 5, 5))
    for m in MODES:
        T, A = orc.correlate(src, w, m)
        for first, last in (((0, 0, 0), (13, 9, 11)), ((0, 0, 0), (3, 2, 4)),
                            ((10, 7, 8), (13, 9, 11)), ((4, 3, 2), (9, 6, 7)),
                            ((5, 5, 5), (5, 9, 11))):
            for nt in (1, 3):
                Tb, Ab = orc.correlate_box(src, w, m, first, last, nthreads=nt)
                sl = tuple(slice(a, b) for a, b in zip(first[::-1], last[::-1]))
                assert np.array_equal(Tb, T[sl]) and np.array_equal(Ab, A[sl]), (m, first)
    with pytest.raises(ValueError):
        orc.correlate_box(src, w, "clamp", (0, 0, 0), (14, 9, 11))


def test_z_range_and_threads(orc):
    g = np.random.default_rng(15)
    src = g.random((10, 6, 7)).astype(np.float32)
    w = g.standard_normal((3, 3, 3))
    full, _ = orc.correlate(src, w, "mirror", nthreads=1)
    part, _ = orc.correlate(src, w, "mirror", z_range=(3, 8), nthreads=4)
    assert np.array_equal(part, full[3:8])


# ------------------------------------------------------------------ fill --

def test_fig4_fill_range_example(orc):
    gold = json.load(open(os.path.join(GOLD, "fig4_fill_range.json")))
    X, Y, Z = gold["dims"]
    vol = np.zeros((Z, Y, X), np.uint8)
    raw = orc.fill_raw(gold["value"], *gold["range"], np.uint8)
    assert raw == gold["expected_raw"]
    orc.fill_range(vol, gold["first"], gold["last"], raw)
    assert int((vol == raw).sum()) == gold["expected_count_raw"]
    assert int((vol == 0).sum()) == gold["expected_count_zero"]
    assert vol[0].max() == 0 and vol[-1].max() == 0
    assert vol[:, :, 0].max() == 0 and vol[:, :, 63].max() == 0
    assert vol[1, 1, 1] == 255 and vol[62, 62, 62] == 255


def test_fill_value_mapping(orc):
    """Worked values of the range mapping: raw = clamp(floor((v - lo) /
    (hi - lo) * max + 1/2), 0, max); float32 stores the value itself."""
    assert orc.fill_raw(0.25, 0, 1, np.uint8) == 64        # 63.75 -> 64
    assert orc.fill_raw(0.0, -1, 1, np.uint16) == 32768    # 32767.5 -> 32768
    assert orc.fill_raw(2.0, 0, 1, np.uint8) == 255
    assert orc.fill_raw(-3.0, 0, 1, np.uint16) == 0
    assert orc.fill_raw(100.0, 0, 255, np.uint8) == 100
    assert orc.fill_raw(-1.5, 0, 1, np.float32) == -1.5
    with pytest.raises(ValueError):
        orc.fill_raw(1.0, 2.0, 2.0, np.uint8)
