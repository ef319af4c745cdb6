"""GPU check of vktApplyFilterBatchedNoAlloc, the allocation-free batched
form: through the C interface, its outputs equal vktApplyFilterBatched's bit
for bit (the same class kernels and slab depths), on two calls in a row, the
second with a smaller batch of smaller volumes (the static scratch array
keeps the first call's contents), and both against the oracle at the stated
tolerances."""
import numpy as np
import pytest

from _gpu import check_against_oracle, sentinel_like, to_device

pytestmark = pytest.mark.gpu


def _vol(g, shape, dtype):
    if dtype == np.float32:
        return g.standard_normal(shape).astype(np.float32)
    return g.integers(0, np.iinfo(dtype).max + 1, shape).astype(dtype)


def _batch(vkt, specs, seed):
    g = np.random.default_rng(seed)
    items = []
    for shape, dtype, k, kind in specs:
        src = _vol(g, shape, dtype)
        if kind == "int":
            w = g.integers(-3, 6, (k, k, k)).astype(np.int32)
            D = int(g.integers(1, 60))
            hf = vkt.vktFilterCreateInt(w, D)
        else:
            w = g.standard_normal((k, k, k)).astype(np.float32)
            if dtype != np.float32:
                w = (np.abs(w) / np.abs(w).sum()).astype(np.float32)
            D = None
            hf = vkt.vktFilterCreate(w)
        s_t = to_device(src)
        a_t, b_t = sentinel_like(s_t), sentinel_like(s_t)
        items.append(dict(src=src, w=w, D=D, hf=hf, s_t=s_t, a_t=a_t, b_t=b_t,
                          hs=vkt.volume_from_tensor(s_t), ha=vkt.volume_from_tensor(a_t),
                          hb=vkt.volume_from_tensor(b_t)))
    return items


FIRST = [((40, 37, 90), np.uint16, 5, "float"), ((17, 70, 33), np.uint16, 7, "float"),
         ((33, 64, 64), np.uint8, 3, "int"), ((20, 41, 132), np.uint8, 5, "int"),
         ((12, 30, 50), np.float32, 5, "float"), ((25, 25, 25), np.float32, 3, "float"),
         ((6, 96, 70), np.float32, 9, "float"), ((5, 129, 40), np.uint16, 3, "int"),
         ((64, 80, 72), np.uint16, 3, "float"), ((3, 2, 1), np.uint16, 5, "float")]
SECOND = [((9, 33, 65), np.uint16, 5, "float"), ((8, 16, 16), np.uint8, 3, "int"),
          ((7, 9, 11), np.float32, 3, "float")]


@pytest.mark.parametrize("mode", ["clamp", "border"])
def test_no_alloc_equals_batched_twice(orc, mode):
    import torch
    from paper_2203_10213_amd import vkt
    vkt.vktSetPrecision("auto")
    vkt.vktSetAutotune(False)
    vkt.vktSetStream(torch.cuda.current_stream())
    batches = [_batch(vkt, FIRST, 21), _batch(vkt, SECOND, 22)]
    try:
        for call, items in enumerate(batches):
            print(f"no-alloc call {call}: {len(items)} volumes, mode {mode}", flush=True)
            vkt.vktApplyFilterBatched([x["ha"] for x in items], [x["hs"] for x in items],
                                      [x["hf"] for x in items], mode)
            vkt.vktApplyFilterBatchedNoAlloc([x["hb"] for x in items], [x["hs"] for x in items],
                                             [x["hf"] for x in items], mode)
            vkt.vktSynchronize()
            for i, x in enumerate(items):
                a = x["a_t"].cpu().numpy()
                b = x["b_t"].cpu().numpy()
                assert np.array_equal(a.view(np.uint8), b.view(np.uint8)), (call, i)
                check_against_oracle(orc, x["src"], x["w"], mode, b, divisor=x["D"],
                                     what=f"no-alloc call {call} item {i}")
    finally:
        for items in batches:
            for x in items:
                vkt.vktFilterDestroy(x["hf"])
                for h in ("hs", "ha", "hb"):
                    vkt.vktStructuredVolumeDestroy(x[h])
        vkt.vktSetStream(None)


def test_no_alloc_rejects_oversized_batch():
    """A batch whose work list cannot fit the static array is refused before
    anything is enqueued (the output keeps its sentinel)."""
    import torch
    from paper_2203_10213_amd import vkt
    vkt.vktSetPrecision("auto")
    vkt.vktSetStream(torch.cuda.current_stream())
    # 8 MiB of 8-byte work items at one item per 64x32x6-cell tile-slab of the
    # vector kernel would need > 8e12 cells; instead use many tiny volumes:
    # each needs one descriptor (> 64 bytes) -- 140000 1-cell volumes exceed it
    n = 140000
    src = torch.zeros(n, dtype=torch.float32, device="cuda")
    dst = torch.full((n,), float("nan"), dtype=torch.float32, device="cuda")
    hf = vkt.vktFilterCreate(np.ones((3, 3, 3), np.float32) / 27)
    hs, hd = [], []
    try:
        for i in range(n):
            hs.append(vkt.vktStructuredVolumeCreateFromDevicePtr(
                (1, 1, 1), vkt.vktDataFormatFloat32, src.data_ptr() + 4 * i))
            hd.append(vkt.vktStructuredVolumeCreateFromDevicePtr(
                (1, 1, 1), vkt.vktDataFormatFloat32, dst.data_ptr() + 4 * i))
        with pytest.raises(vkt.VktError) as e:
            vkt.vktApplyFilterBatchedNoAlloc(hd, hs, [hf] * n)
        assert e.value.code == vkt.vktUnsupported
        torch.cuda.synchronize()
        assert torch.isnan(dst).all()
    finally:
        for h in hs + hd:
            vkt.vktStructuredVolumeDestroy(h)
        vkt.vktFilterDestroy(hf)
        vkt.vktSetStream(None)
