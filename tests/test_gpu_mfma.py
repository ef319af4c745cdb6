"""GPU parity of the matrix-core (split 16-bit operand) ApplyFilter path.

Float-weight filters with k >= 5 run on the matrix cores unless the thread's
precision is FP32.  Tolerances: integer cells within 1 LSB of the oracle's
stored result; float32 cells within 1e-5 of sum |w||s| (both the 3- and the
6-product split), the 6-product split within 1e-6.
"""
import numpy as np
import pytest

from _gpu import check_against_oracle, run_filter

pytestmark = pytest.mark.gpu

MODES = ["clamp", "wrap", "mirror", "border"]
KS = [5, 7, 9, 11, 13, 15]
# (Z, Y, X): several 32x64 output tiles with ragged tails, small and tiny axes
SHAPES = [(3, 2, 1), (9, 70, 33), (21, 65, 70), (6, 130, 97)]


def _vol(g, shape, dtype):
    if dtype == np.float32:
        return g.standard_normal(shape).astype(np.float32)
    return g.integers(0, np.iinfo(dtype).max + 1, shape).astype(dtype)


@pytest.fixture(autouse=True)
def _reset_precision():
    from paper_2203_10213_amd import vkt
    rp = vkt.vktGetRowPairMinCells()
    yield
    vkt.vktSetPrecision("auto")
    vkt.vktSetRowPairMinCells(rp)


@pytest.mark.parametrize("precision", ["splitbf16", "splitbf16x6"])
@pytest.mark.parametrize("dtype", [np.uint8, np.uint16, np.float32])
@pytest.mark.parametrize("mode", ["clamp", "wrap", "border"])
def test_row_pair_kernel_forced(orc, precision, dtype, mode):
    """The row-pair kernel (k = 5, and 3-product float32 k = 7) on small,
    ragged volumes: the row-pair threshold at 0 cells sends every such job
    there; the other jobs keep their 16x16x32 path."""
    from paper_2203_10213_amd import vkt
    vkt.vktSetRowPairMinCells(0)
    g = np.random.default_rng(350 + MODES.index(mode))
    for shape in SHAPES:
        for k in (5, 7):
            src = _vol(g, shape, dtype)
            w = g.standard_normal((k, k, k)).astype(np.float32)
            if dtype != np.float32:
                w = np.abs(w) / np.abs(w).sum()
            out = run_filter(src, w, mode, precision=precision)
            check_against_oracle(orc, src, w, mode, out,
                                 tol=1e-6 if (precision == "splitbf16x6"
                                              and dtype == np.float32) else 1e-5,
                                 what=f"row pairs {precision} {shape} k={k}")


@pytest.mark.parametrize("precision", ["splitbf16", "splitbf16x6"])
@pytest.mark.parametrize("dtype", [np.uint8, np.uint16, np.float32])
@pytest.mark.parametrize("mode", MODES)
def test_split_sweep(orc, precision, dtype, mode):
    g = np.random.default_rng(300 + MODES.index(mode) + 10 * KS.index(5))
    worst = 0.0
    for shape in SHAPES:
        for k in KS:
            if np.prod(shape) * k ** 3 > 8e7:
                continue
            src = _vol(g, shape, dtype)
            w = g.standard_normal((k, k, k)).astype(np.float32)
            if dtype != np.float32:
                w = np.abs(w) / np.abs(w).sum()
            out = run_filter(src, w, mode, precision=precision)
            e = check_against_oracle(orc, src, w, mode, out,
                                     tol=1e-6 if (precision == "splitbf16x6"
                                                  and dtype == np.float32) else 1e-5,
                                     what=f"{precision} {shape} k={k}")
            worst = max(worst, e)
    print(f"{precision} {np.dtype(dtype).name} {mode}: worst error {worst:.3g}")


def test_split_matches_plain_on_gaussians(orc):
    """Mixed-sign edge-detection-like and Gaussian filters on a float32
    volume: split (3 products) stays within 1e-5 of sum |w||s|."""
    from paper_2203_10213_amd import synth
    g = np.random.default_rng(9)
    src = (g.random((24, 96, 80)) * 1000).astype(np.float32)
    for k in (5, 7, 9, 11):
        w = synth.gaussian_weights(k, k / 4)
        lap = -w.copy()
        lap[k // 2, k // 2, k // 2] += 1.0  # identity minus blur: signed weights
        for ww in (w, lap.astype(np.float32)):
            out = run_filter(src, ww, "clamp", precision="splitbf16")
            check_against_oracle(orc, src, ww, "clamp", out, what=f"k={k}")


@pytest.mark.parametrize("dtype", [np.uint8, np.uint16, np.float32])
def test_split_delta_identity(dtype):
    """A centred delta reproduces the input: exactly for integer cells; for
    float32 within the split's resolution (6 products: exactly)."""
    g = np.random.default_rng(4)
    src = _vol(g, (9, 70, 40), dtype)
    for k in (5, 9, 11):
        w = np.zeros((k, k, k), np.float32)
        w[k // 2, k // 2, k // 2] = 1.0
        out = run_filter(src, w, "clamp", precision="splitbf16x6")
        assert np.array_equal(out, src), k
        out3 = run_filter(src, w, "clamp", precision="splitbf16")
        if dtype == np.float32:
            rel = np.abs(out3.astype(np.float64) - src) / np.maximum(np.abs(src), 1e-30)
            assert rel.max() <= 2.0 ** -16
        else:
            assert np.array_equal(out3, src)


def test_fp32_precision_forces_vector_path(orc):
    """precision fp32 keeps k >= 5 on the FP32 vector path: results agree with
    the split path within tolerance but come from a different arithmetic."""
    g = np.random.default_rng(2)
    src = _vol(g, (10, 40, 50), np.float32)
    w = g.standard_normal((7, 7, 7)).astype(np.float32)
    a = run_filter(src, w, "clamp", precision="fp32")
    b = run_filter(src, w, "clamp", precision="splitbf16")
    check_against_oracle(orc, src, w, "clamp", a)
    check_against_oracle(orc, src, w, "clamp", b)
    assert not np.array_equal(a, b)


def test_c3_blob_field_dense7_dense9_blocks(orc):
    """1024^3 float32 blob field, dense 7^3 and 9^3 unit-L1 weights: both
    split variants and the plain FP32 form against the oracle on every cell
    of 520 32^3 blocks (the 8 corner blocks and 512 uniformly placed ones),
    within 1e-5 of sum |w||s| (6 products: 1e-6); max and RMS errors are
    printed per result."""
    import torch
    from paper_2203_10213_amd import synth, vkt
    from _gpu import device_blocks, float_error_stats, oracle_blocks
    src_t = synth.blob_field_f32(1024, 64, synth.SEEDS["c3"], device="cuda")
    src = src_t.cpu().numpy()
    origins = synth.sample_blocks(src.shape, 512, synth.SEEDS["c3_blocks"])
    dst_t = torch.empty_like(src_t)
    for k, seed in ((7, synth.SEEDS["c3a_w"]), (9, synth.SEEDS["c3b_w"])):
        w = synth.random_l1(k, seed)
        T, A = oracle_blocks(orc, src, w, "clamp", origins)
        for prec, tol in (("splitbf16", 1e-5), ("splitbf16x6", 1e-6), ("fp32", 1e-5)):
            dst_t.fill_(float("nan"))
            vkt.vktSetPrecision(prec)
            vkt.apply_filter(dst_t, src_t, w, "clamp")
            torch.cuda.synchronize()
            got = device_blocks(dst_t, origins)
            st = float_error_stats(got, T, A)
            print(f"C3 k={k} {prec}: max |gpu-T| {st['max_abs']:.3g} rms {st['rms_abs']:.3g}; "
                  f"max e {st['max_rel']:.3g} rms e {st['rms_rel']:.3g}")
            assert st["max_rel"] <= tol, (k, prec, st)
    del src_t, dst_t
    torch.cuda.empty_cache()


def test_c5_ellipsoid_u16_gauss11_subblocks(orc):
    """2048 x 2048 x 1024 uint16 ellipsoid phantom, 11^3 Gaussian sigma 2.5
    on the split path and on the rank-1 form: 64 32^3 sub-blocks (the 8
    corner blocks and 56 random ones) checked cell by cell, within 1 LSB."""
    import torch
    from paper_2203_10213_amd import synth, vkt
    src_t = synth.ellipsoid_phantom_u16((1024, 2048, 2048), 5000, synth.SEEDS["c5"],
                                        device="cuda")
    assert src_t.dtype == torch.uint16
    w = synth.gaussian_weights(11, 2.5)
    dst_t = torch.empty_like(src_t)
    vkt.vktSetPrecision("splitbf16")
    vkt.apply_filter(dst_t, src_t, w, "clamp")
    # the rank-1 form of the same (separable) filter, on the same blocks
    sep_t = torch.empty_like(src_t)
    vkt.vktSetSeparable(True)
    try:
        vkt.apply_filter(sep_t, src_t, w, "clamp")
    finally:
        vkt.vktSetSeparable(False)
    torch.cuda.synchronize()
    Z, Y, X = src_t.shape
    g = np.random.default_rng(synth.SEEDS["c5_blocks"])
    corners = [(x, y, z) for x in (0, X - 32) for y in (0, Y - 32) for z in (0, Z - 32)]
    rand = [(int(g.integers(0, X - 31)), int(g.integers(0, Y - 31)), int(g.integers(0, Z - 31)))
            for _ in range(56)]
    r = 5
    for (bx, by, bz) in corners + rand:
        # the block plus its clamped halo, copied out of the device volume
        zs = np.clip(np.arange(bz - r, bz + 32 + r), 0, Z - 1)
        ys = np.clip(np.arange(by - r, by + 32 + r), 0, Y - 1)
        xs = np.clip(np.arange(bx - r, bx + 32 + r), 0, X - 1)
        idx = torch.from_numpy(zs).cuda(), torch.from_numpy(ys).cuda(), torch.from_numpy(xs).cuda()
        sub = src_t.view(torch.int16)[idx[0]][:, idx[1]][:, :, idx[2]].cpu().numpy().view(np.uint16)
        T, _ = orc.correlate(sub, w.astype(np.float64), "clamp")  # halo makes clamp exact
        want = orc.store_float_filter(T[r:-r, r:-r, r:-r], np.uint16)
        for name, out_t in (("split", dst_t), ("rank-1", sep_t)):
            got = out_t.view(torch.int16)[bz:bz + 32, by:by + 32, bx:bx + 32].cpu().numpy()
            diff = np.abs(got.view(np.uint16).astype(np.int64) - want.astype(np.int64))
            assert diff.max() <= 1, (name, bx, by, bz, diff.max())
    del src_t, dst_t, sep_t
    torch.cuda.empty_cache()
