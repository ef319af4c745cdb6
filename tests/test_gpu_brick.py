"""GPU parity of vktBrickDecompose (paper Sec. 3.2, domain decomposition:
bricks with optional ghost cells): every brick bit-exact against the
oracle's brick_decompose for every format and address mode, with ragged
last bricks, ghosts wider than bricks or than the volume, and more bricks
than one launch carries; and bricks with ghosts of the filter radius,
filtered together by vktApplyFilterBatched, reproduce the whole-volume
ApplyFilter on their interiors (oracle tolerances)."""
import numpy as np
import pytest

from _gpu import check_against_oracle, to_device

pytestmark = pytest.mark.gpu

MODES = ["clamp", "wrap", "mirror", "border"]
DTYPES = [np.uint8, np.uint16, np.float32]


def _vol(g, shape, dtype):
    if dtype == np.float32:
        return g.standard_normal(shape).astype(np.float32)
    return g.integers(0, np.iinfo(dtype).max + 1, shape).astype(dtype)


CASES = [  # (Z, Y, X), brick (x, y, z), ghost (x, y, z)
    ((9, 20, 33), (16, 8, 4), (1, 1, 1)),
    ((5, 6, 7), (2, 2, 2), (3, 3, 3)),          # ghosts wider than bricks
    ((3, 4, 2), (8, 8, 8), (2, 1, 4)),          # one brick, ghosts beyond the volume
    ((8, 2, 300), (100, 1, 3), (0, 5, 2)),      # rows wider than a block
    ((10, 20, 30), (2, 2, 2), (1, 0, 1)),       # 750 bricks: several launches
    # rows of whole dwords (the row kernel; every float32 case): source
    # dwords straddled at a 2-byte offset, x faces inside the first and last
    # dword of a row
    ((6, 10, 64), (16, 4, 3), (2, 1, 1)),
    ((5, 7, 40), (8, 3, 2), (4, 2, 1)),         # aligned, faces
    ((4, 5, 12), (12, 2, 2), (2, 0, 1)),        # one brick along x
    # uint16 rows of whole dwords at a 2-byte source offset (odd ghost width)
    ((6, 9, 50), (10, 3, 4), (3, 1, 2)),
    ((3, 5, 8), (8, 5, 3), (6, 0, 0)),          # rows with fewer than 4 inside dwords
]


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("dtype", DTYPES)
def test_bricks_match_oracle(orc, dtype, mode):
    from paper_2203_10213_amd import vkt
    g = np.random.default_rng(830 + DTYPES.index(dtype) * 4 + MODES.index(mode))
    for shape, brick, ghost in CASES:
        src = _vol(g, shape, dtype)
        got = vkt.brick_decompose(to_device(src), brick, ghost, mode)
        vkt.vktSynchronize()
        want = orc.brick_decompose(src, brick, ghost, mode)
        assert len(got) == len(want)
        for i, (a, b) in enumerate(zip(got, want)):
            a = a.cpu().numpy()
            assert a.shape == b.shape and np.array_equal(a.view(np.uint8), b.view(np.uint8)), \
                f"{dtype.__name__} {mode} {shape} brick {brick} ghost {ghost}: brick {i}"


def _stitch(bricks, shape, brick, r):
    Z, Y, X = shape
    BX, BY, BZ = brick
    nbx, nby = -(-X // BX), -(-Y // BY)
    out = np.empty(shape, bricks[0].dtype)
    for i, b in enumerate(bricks):
        bx, by, bz = i % nbx, (i // nbx) % nby, i // (nbx * nby)
        inner = b[r:b.shape[0] - r, r:b.shape[1] - r, r:b.shape[2] - r]
        out[bz * BZ:bz * BZ + inner.shape[0], by * BY:by * BY + inner.shape[1],
            bx * BX:bx * BX + inner.shape[2]] = inner
    return out


@pytest.mark.parametrize("mode", MODES)
def test_ghosted_bricks_feed_the_batched_filter(orc, mode):
    """Decompose with ghosts r, filter all bricks in one batched call (mode
    border: never reached by the interiors), stitch the interiors back."""
    import torch
    from paper_2203_10213_amd import synth, vkt
    g = np.random.default_rng(850 + MODES.index(mode))
    for dtype, w, D, shape, brick in [
            (np.uint16, synth.gaussian_weights(5, 1.25), None, (40, 70, 90), (32, 32, 16)),
            (np.float32, g.standard_normal((7, 7, 7)).astype(np.float32), None, (30, 45, 50),
             (24, 20, 12)),
            (np.uint8, np.ones((3, 3, 3), np.int32), 27, (20, 33, 70), (64, 16, 8))]:
        src = _vol(g, shape, dtype)
        r = w.shape[0] // 2
        bricks = vkt.brick_decompose(to_device(src), brick, (r, r, r), mode)
        outs = [torch.empty_like(b) for b in bricks]
        hs = [vkt.volume_from_tensor(b) for b in bricks]
        hd = [vkt.volume_from_tensor(o) for o in outs]
        hf = vkt.vktFilterCreate(w) if D is None else vkt.vktFilterCreateInt(w, D)
        try:
            vkt.vktSetStream(torch.cuda.current_stream())
            vkt.vktSetPrecision("auto")
            vkt.vktApplyFilterBatched(hd, hs, [hf] * len(hs), "border")
            vkt.vktSynchronize()
        finally:
            vkt.vktFilterDestroy(hf)
            for h in hs + hd:
                vkt.vktStructuredVolumeDestroy(h)
        got = _stitch([o.cpu().numpy() for o in outs], shape, brick, r)
        check_against_oracle(orc, src, w, mode, got, divisor=D,
                             what=f"bricks {dtype.__name__} k={w.shape[0]} {mode}")


def test_invalid_arguments():
    import torch
    from paper_2203_10213_amd import vkt
    src = torch.zeros((4, 6, 8), dtype=torch.uint16, device="cuda")
    hs = vkt.volume_from_tensor(src)
    assert vkt.vktBrickDecomposeGetNumBricks(hs, (3, 4, 4)) == (3, 2, 1)
    assert vkt.vktBrickDecomposeGetBrickDims(hs, (3, 4, 4), (1, 2, 0), (2, 1, 0)) == (4, 6, 4)
    tens = [torch.zeros((4, 8, 5), dtype=torch.uint16, device="cuda") for _ in range(6)]
    hb = [vkt.volume_from_tensor(t) for t in tens]
    # bricks (4, 3, 4) with ghost y 1: 2 x 2 x 1 bricks of 4 x 5 x 4 cells
    quads = [torch.zeros((4, 5, 4), dtype=torch.uint16, device="cuda") for _ in range(4)]
    hq = [vkt.volume_from_tensor(t) for t in quads]
    odd = torch.zeros((4, 5, 4), dtype=torch.uint8, device="cuda")
    ho = vkt.volume_from_tensor(odd)
    try:
        bad = [lambda: vkt.vktBrickDecomposeGetNumBricks(hs, (0, 1, 1)),
               lambda: vkt.vktBrickDecomposeGetBrickDims(hs, (3, 4, 4), (0, 0, 0), (3, 0, 0)),
               lambda: vkt.vktBrickDecomposeGetBrickDims(hs, (3, 4, 4), (-1, 0, 0), (0, 0, 0)),
               lambda: vkt.vktBrickDecompose(hb[:5], hs, (3, 4, 4), (1, 2, 0)),   # count
               lambda: vkt.vktBrickDecompose(hb, hs, (3, 4, 4), (1, 2, 0)),       # dims
               lambda: vkt.vktBrickDecompose([hq[0]] * 4, hs, (4, 3, 4), (0, 1, 0)),  # overlap
               lambda: vkt.vktBrickDecompose([ho] + hq[1:], hs, (4, 3, 4), (0, 1, 0)),  # format
               lambda: vkt.vktBrickDecompose(hq, hs, (4, 3, 4), (0, 1, 0), 9)]    # mode
        for call in bad:
            with pytest.raises(vkt.VktError) as e:
                call()
            assert e.value.code == vkt.vktInvalidValue
        vkt.vktBrickDecompose(hq, hs, (4, 3, 4), (0, 1, 0))
        vkt.vktSynchronize()
        # 8 x 6 x 4 with bricks (4, 3, 4) and ghost y 1: 2 x 2 x 1 bricks of 4 x 5 x 4
        assert vkt.vktBrickDecomposeGetBrickDims(hs, (4, 3, 4), (0, 1, 0), (1, 1, 0)) == (4, 5, 4)
    finally:
        for h in hb + hq + [hs, ho]:
            vkt.vktStructuredVolumeDestroy(h)


def test_512_uint8_into_64_bricks_with_2_ghosts(orc):
    """The 512^3 uint8 phantom into 64^3 bricks with 2 ghost cells under
    clamp (512 bricks, one launch), every brick bit-exact."""
    from paper_2203_10213_amd import synth, vkt
    src = synth.ct_phantom_u8(512, synth.SEEDS["c2a"])
    got = vkt.brick_decompose(to_device(src), (64, 64, 64), (2, 2, 2), "clamp")
    vkt.vktSynchronize()
    want = orc.brick_decompose(src, (64, 64, 64), (2, 2, 2), "clamp")
    assert len(got) == len(want) == 512
    for i, (a, b) in enumerate(zip(got, want)):
        assert np.array_equal(a.cpu().numpy(), b), f"brick {i}"
