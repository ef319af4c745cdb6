"""Throughput benchmark of vktApplyFilter on one MI355X.

Default workload: the plain-path pair of 512^3 volumes --
  (a) uint8 CT-like phantom (N(40, 8^2) background, 200 solid spheres),
      integer 3^3 box filter with divisor 27, clamp, uint8 out (bit-exact);
  (b) float32 smoothed Gaussian noise (sigma 4), 5^3 Gaussian sigma 1.5,
      clamp, float32 out.
One step = one ApplyFilter of (a) and one of (b), with inputs resident in HBM.
Prints ONE JSON line (metric Gvoxels/s = output cells / device time).

Other workloads (--workload): c1 (64^3 float32, 3^3 Gaussian), c3a / c3b
(1024^3 float32 blob field, dense 7^3 / 9^3 unit-L1 weights), c4 (256 uneven
uint16 volumes, batched), c5 (2048 x 2048 x 1024 uint16 ellipsoid phantom,
11^3 Gaussian sigma 2.5), transforms (the two 512^3 volumes of the default
workload: Resample down by two on every axis and Flip along the longest
axis, the paper's other structured-volume benchmarks).
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
FP32_VECTOR_PEAK_TF = 157.3    # MI355X FP32 vector (packed FMA), TFLOP/s
BF16_MFMA_PEAK_TF = 2500.0     # MI355X dense bf16 matrix, TFLOP/s
# 8-bit dot products on the vector ALUs: 256 CUs x 4 SIMDs x 16 lanes x 4 MACs
# x 2 ops x 2.4 GHz (v_dot4 issues at the full VALU rate)
INT8_DOT_PEAK_TOPS = 256 * 4 * 16 * 4 * 2 * 2.4e9 / 1e12
INT8_MFMA_PEAK_TOPS = 5000.0   # MI355X dense int8 matrix, TOP/s


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="c2",
                    choices=["c1", "c2", "c2a", "c2b", "c3a", "c3b", "c4", "c5",
                             "transforms"])
    ap.add_argument("--precision", default=None,
                    choices=["auto", "fp32", "splitbf16", "splitbf16x6"],
                    help="default: fp32 for c1/c2 (the plain-path configurations), "
                         "auto (split bf16/fp16 matrix path for k >= 5) otherwise")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--int8-matrix", action="store_true",
                    help="uint8 3^3 integer filters on the int8 matrix cores instead of "
                         "the 8-bit dot products (vktSetInt8Matrix(1))")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target CPU time of the oracle baseline sample")
    ap.add_argument("--separable", action="store_true",
                    help="rank-1 fast path (vktSetSeparable): three 1-D passes for separable "
                         "filters; reported apart from the dense numbers")
    ap.add_argument("--autotune", action="store_true",
                    help="c4: let the batched planner time its slab-depth candidates")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device copy (counter calibration)")
    return ap.parse_args()


# --------------------------------------------------------------- workloads --

def make_cases(name, device):
    """List of dicts: name, src tensor, weights, divisor, flops/voxel, bytes."""
    import numpy as np
    import torch
    from paper_2203_10213_amd import synth
    S = synth.SEEDS
    cases = []
    if name in ("c2", "c2a"):
        src = torch.from_numpy(synth.ct_phantom_u8(512, S["c2a"])).to(device)
        w, D = synth.box_int(3)
        cases.append(dict(name="c2a_u8_512_box3_div27", src=src, w=w, D=D, k=3))
    if name in ("c2", "c2b"):
        src = synth.smoothed_noise_f32(512, 4.0, S["c2b"], device=device)
        cases.append(dict(name="c2b_f32_512_gauss5_s1.5", src=src,
                          w=synth.gaussian_weights(5, 1.5), D=None, k=5))
    if name == "c1":
        src = torch.from_numpy(synth.uniform_f32((64, 64, 64), S["c1"])).to(device)
        cases.append(dict(name="c1_f32_64_gauss3_s1", src=src,
                          w=synth.gaussian_weights(3, 1.0), D=None, k=3))
    if name in ("c3a", "c3b"):
        k = 7 if name == "c3a" else 9
        src = synth.blob_field_f32(1024, 64, S["c3"], device=device)
        w = synth.random_l1(k, S["c3a_w"] if k == 7 else S["c3b_w"])
        cases.append(dict(name=f"{name}_f32_1024_dense{k}_l1", src=src, w=w, D=None, k=k))
    if name == "c5":
        src = synth.ellipsoid_phantom_u16((1024, 2048, 2048), 5000, S["c5"], device=device)
        cases.append(dict(name="c5_u16_2048x2048x1024_gauss11_s2.5", src=src,
                          w=synth.gaussian_weights(11, 2.5), D=None, k=11))
    for c in cases:
        c["voxels"] = c["src"].numel()
        c["cell_bytes"] = c["src"].element_size()
        c["flops_per_voxel"] = 2 * c["k"] ** 3
    return cases


KERNEL_SOURCES = {
    "resample": ["vkt_resample.hip", "vkt_internal.h"],
    "valu": ["vkt_filter_valu.hip", "vkt_internal.h"],
    "dot4": ["vkt_filter_dot4.hip", "vkt_internal.h"],
    "i8mma": ["vkt_filter_i8mma.hip", "vkt_internal.h"],
    "mfma": ["vkt_filter_mfma.hip", "vkt_internal.h"],
}


def kernel_source_sha(path):
    """Hash of the HIP sources of one kernel path; profile-derived traffic is
    only reported for the kernel it was measured on."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2203_10213_amd", "csrc")
    for f in KERNEL_SOURCES[path]:
        p = os.path.join(csrc, f)
        if os.path.exists(p):
            h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def stored_traffic(case_name, path):
    """HBM bytes per launch from committed rocprofv3 --pmc summaries, scaled
    by the copy-kernel calibration, if they match the current kernel."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
        e = d.get(case_name)
        if e and e.get("path") == path and e.get("kernel_src_sha") == kernel_source_sha(path):
            return e["hbm_bytes_per_launch"]
    except (ValueError, KeyError):
        pass
    return None


def arith_dtype(c, precision):
    """The type the path computes in."""
    if c["path"] == "mfma":
        if c["src"].dtype.is_floating_point:
            return "bf16x3->f32" if precision == "splitbf16" else "bf16x6->f32"
        return "f16x2->f32"
    if c["path"] == "dot4":
        return "u8dot4->i32"
    if c["path"] == "i8mma":
        return "i8mma->i32"
    if c["path"] == "sep":
        return "f32(rank-1)"
    if c["D"] is not None:
        return "f32(exact int)"
    return "f32"


def kernel_path(c, precision, separable=False, int8_matrix=False):
    """The library's plan rule: float-weight filters with k >= 5 run on the
    matrix cores unless the precision is fp32; uint8 volumes with integer
    filters of k <= 7, weights all in [0, 255] or all in [-128, 127],
    sum |w| <= 2048, divisor <= 2^19 and rows of a multiple of 4 cells run as
    8-bit dot products (k = 3 with weights in [-128, 127] as int8 products on
    the matrix cores when that is turned on); the rest on the vector ALUs in
    FP32 / int32."""
    import numpy as np
    if separable and rank1(c["w"]) and not (c["k"] <= 3 and dot4_ok(c)):
        return "sep"
    if c["D"] is None:
        return "mfma" if (c["k"] >= 5 and precision != "fp32") else "valu"
    if not dot4_ok(c):
        return "valu"
    w = np.asarray(c["w"], np.int64)
    if int8_matrix and c["k"] == 3 and w.min() >= -128 and w.max() <= 127:
        return "i8mma"
    return "dot4"


def dot4_ok(c):
    """The 8-bit dot-product path's eligibility (uint8 cells, integer
    filter, k <= 7, weights in [0, 255] or [-128, 127], sum |w| <= 2048,
    divisor <= 2^19, rows of a multiple of 4 cells)."""
    import numpy as np
    if c["D"] is None:
        return False
    w = np.asarray(c["w"], np.int64)
    fits = (w.min() >= 0 and w.max() <= 255) or (w.min() >= -128 and w.max() <= 127)
    return bool(c["src"].dtype == torch_uint8() and c["k"] in (3, 5, 7) and fits
                and np.abs(w).sum() <= 2048 and c["D"] <= (1 << 19)
                and c["src"].shape[-1] % 4 == 0)


def rank1(w):
    """The library's rank-1 test (float filters to 2^-21 max|w|; the integer
    filters of these workloads are exact outer products)."""
    import numpy as np
    w = np.asarray(w, np.float64)
    k = w.shape[0]
    ip = np.unravel_index(np.argmax(np.abs(w)), w.shape)
    p = w[ip]
    if p == 0:
        return False
    t, v, u = w[:, ip[1], ip[2]] / p, w[ip[0], :, ip[2]] / p, w[ip[0], ip[1], :]
    return bool(np.max(np.abs(np.einsum("c,b,a->cba", t, v, u) - w)) <= np.ldexp(abs(p), -21))


def torch_uint8():
    import torch
    return torch.uint8


def case_roofline(c, ms):
    """Algorithmic bytes (1 cell read + 1 cell written per output) and flops
    (2 k^3 per output) over the measured time, against the roofline that
    bounds this path: HBM, the FP32 vector ALUs, or the dense 16-bit matrix
    cores (split products and Toeplitz zeros are overhead, not counted)."""
    t = ms * 1e-3
    bytes_alg = 2 * c["voxels"] * c["cell_bytes"]
    # the rank-1 path's algorithm is three 1-D passes: 2 * 3k flops per output
    flops = c["voxels"] * (6 * c["k"] if c.get("path") == "sep" else c["flops_per_voxel"])
    gbs = bytes_alg / t / 1e9
    tfs = flops / t / 1e12
    peak_c = {"mfma": BF16_MFMA_PEAK_TF, "dot4": INT8_DOT_PEAK_TOPS,
              "i8mma": INT8_MFMA_PEAK_TOPS}.get(c["path"], FP32_VECTOR_PEAK_TF)
    if bytes_alg / (HBM_PEAK_GBS * 1e9) >= flops / (peak_c * 1e12):
        roof = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": gbs / HBM_PEAK_GBS}
    else:
        roof = {"bound": "mfma" if c["path"] in ("mfma", "i8mma") else "alu", "achieved": tfs,
                "peak": peak_c,
                "unit": "TOP/s" if c["path"] in ("dot4", "i8mma") else "TFLOP/s",
                "frac": tfs / peak_c}
    return dict(case=c["name"], path=c["path"], ms=ms,
                gvoxels_s=c["voxels"] / t / 1e9, hbm_gbs=gbs, hbm_frac=gbs / HBM_PEAK_GBS,
                tflops=tfs, algorithmic_bytes=bytes_alg, flops=flops, roofline=roof)


# ------------------------------------------------------------ CPU baseline --

def cpu_baseline(cases, target_s):
    """The FP64 oracle timed on this host's cores on a bounded z-slab of each
    case (same planes count fraction for every case), scaled to Gvoxels/s of
    the whole step's mix."""
    import numpy as np
    import oracle
    nthreads = min(16, os.cpu_count() or 1)
    # calibrate with one plane per case, then size the slab to ~target_s
    per_plane = []
    hosts = []
    for c in cases:
        src = c["src"].cpu().numpy()
        hosts.append(src)
        t0 = time.perf_counter()
        oracle.correlate(src, np.asarray(c["w"], np.float64), "clamp", z_range=(0, 1),
                         nthreads=nthreads, with_abs=False)
        per_plane.append(time.perf_counter() - t0)
    nplanes = max(1, int(target_s / max(sum(per_plane), 1e-6)))
    tot_vox, tot_t = 0, 0.0
    for c, src in zip(cases, hosts):
        Z = src.shape[0]
        z0 = Z // 2
        z1 = min(Z, z0 + nplanes)
        t0 = time.perf_counter()
        oracle.correlate(src, np.asarray(c["w"], np.float64), "clamp", z_range=(z0, z1),
                         nthreads=nthreads, with_abs=False)
        dt = time.perf_counter() - t0
        # weight each case by its share of the step's voxels
        frac = c["voxels"] / (src.shape[1] * src.shape[2] * (z1 - z0))
        tot_vox += c["voxels"]
        tot_t += dt * frac
    return {"value": tot_vox / tot_t / 1e9, "unit": "Gvoxels/s", "cores": nthreads,
            "kind": "oracle",
            "sample": f"FP64 direct-sum oracle on {nplanes} middle z-planes of each case "
                      f"({', '.join(c['name'] for c in cases)}), {nthreads} threads, "
                      f"time scaled to the full volumes"}


# -------------------------------------------------------------------- main --

def copy_probe():
    import torch
    n = 1 << 30
    a = torch.empty(n, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": n, "launches": 3}))


def run_batched(args, vkt, torch):
    """The batched workload: 256 uint16 volumes of uneven sizes, k in {3,5,7}
    Gaussians, one vktApplyFilterBatched (persistent kernels, replayed
    hipGraph) per step; the same work as 256 single launches is timed beside
    it.  Returns the bench line."""
    from paper_2203_10213_amd import synth
    vols, ks = synth.gamma_u16_volumes(256, synth.SEEDS["c4"])
    filts = {k: vkt.vktFilterCreate(synth.gaussian_weights(k, k / 4)) for k in (3, 5, 7)}
    srcs = [torch.from_numpy(v).cuda() for v in vols]
    dsts = [torch.empty_like(x) for x in srcs]
    hs = [vkt.volume_from_tensor(x) for x in srcs]
    hd = [vkt.volume_from_tensor(x) for x in dsts]
    hf = [filts[k] for k in ks]
    stream = torch.cuda.current_stream()
    vkt.vktSetAutotune(args.autotune)
    torch.cuda.synchronize()

    def batched():
        vkt.vktApplyFilterBatched(hd, hs, hf, "clamp")

    def singles():
        for i in range(len(hs)):
            vkt.vktApplyFilter(hd[i], hs[i], hf[i], vkt.vktAddressModeClamp)

    def timed(fn, K, W):
        for _ in range(W):
            fn()
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record(stream)
        for _ in range(K):
            fn()
        t1.record(stream)
        torch.cuda.synchronize()
        return t0.elapsed_time(t1) / K

    print(f"[bench] c4 batched, warmup {args.warmup}", file=sys.stderr, flush=True)
    ms_b = timed(batched, args.steps, args.warmup)
    print("[bench] c4 single launches", file=sys.stderr, flush=True)
    ms_s = timed(singles, max(1, args.steps // 2), 1)
    voxels = sum(int(v.size) for v in vols)
    flops = sum(int(v.size) * 2 * k ** 3 for v, k in zip(vols, ks))
    bytes_alg = 4 * voxels
    t = ms_b * 1e-3
    # the step's binding roofline: the split-fp16 matrix path carries the
    # k = 5, 7 volumes (most of the flops); all volumes move 4 bytes per cell
    mfma_flops = sum(int(v.size) * 2 * k ** 3 for v, k in zip(vols, ks) if k >= 5)
    roof = {"bound": "mfma", "achieved": mfma_flops / t / 1e12, "peak": BF16_MFMA_PEAK_TF,
            "unit": "TFLOP/s", "frac": mfma_flops / t / 1e12 / BF16_MFMA_PEAK_TF,
            "traffic": None, "kernel_case": "c4 k>=5 classes (one graph launch)"}
    line = {
        "metric": "Gvoxels/s ApplyFilter on 1 MI355X",
        "value": voxels / t / 1e9, "unit": "Gvoxels/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_b, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f16x2->f32+f32",
        "data": "synthetic",
        "config": {"workload": "c4", "cases": ["256 u16 volumes, axes U{32..256}, "
                                               "Gaussian k in {3,5,7}, sigma k/4"],
                   "address_mode": "clamp", "precision": args.precision,
                   "autotune": bool(args.autotune)},
        "roofline": roof,
        "cpu_baseline": None,
        "per_case": [{"case": "c4_batched_graph", "ms": ms_b, "gvoxels_s": voxels / t / 1e9,
                      "hbm_frac": bytes_alg / t / 1e9 / HBM_PEAK_GBS, "tflops": flops / t / 1e12},
                     {"case": "c4_256_single_launches", "ms": ms_s,
                      "gvoxels_s": voxels / (ms_s * 1e-3) / 1e9,
                      "hbm_frac": bytes_alg / (ms_s * 1e-3) / 1e9 / HBM_PEAK_GBS,
                      "tflops": flops / (ms_s * 1e-3) / 1e12}],
    }
    for h in hs + hd:
        vkt.vktStructuredVolumeDestroy(h)
    for f in filts.values():
        vkt.vktFilterDestroy(f)
    return line


def run_transforms(args, vkt, torch):
    """Resample by one half on every axis and Flip along the longest axis
    (x for these cubes: the first of the equal extents) of the 512^3 uint8
    phantom and the 512^3 float32 noise field; one step = the four calls.
    Value: source voxels per second over the step.  Flips along y and z and
    BrickDecompose into 64^3 bricks with 2-cell ghosts are timed apart
    (per_case)."""
    import numpy as np
    from paper_2203_10213_amd import synth
    S = synth.SEEDS
    vols = [("u8_512_phantom", torch.from_numpy(synth.ct_phantom_u8(512, S["c2a"])).cuda()),
            ("f32_512_noise", synth.smoothed_noise_f32(512, 4.0, S["c2b"], device="cuda"))]
    stream = torch.cuda.current_stream()
    ops, handles = [], []
    for name, src in vols:
        Z, Y, X = src.shape
        half = torch.empty((Z // 2, Y // 2, X // 2), dtype=src.dtype, device=src.device)
        flipped = torch.empty_like(src)
        hs, hh, hf = (vkt.volume_from_tensor(t) for t in (src, half, flipped))
        handles += [hs, hh, hf]
        n, cb = src.numel(), src.element_size()
        longest = int(np.argmax([X, Y, Z]))
        ops.append(dict(case=f"resample_half_{name}", fn=lambda hh=hh, hs=hs: vkt.vktResample(hh, hs),
                        voxels=n, bytes=n * cb + half.numel() * cb, step=True))
        for ax in (longest,) + tuple(a for a in range(3) if a != longest):
            ops.append(dict(case=f"flip_{'xyz'[ax]}_{name}",
                            fn=lambda hf=hf, hs=hs, ax=ax: vkt.vktFlip(hf, hs, ax),
                            voxels=n, bytes=2 * n * cb, step=ax == longest))
        # BrickDecompose into 64^3 bricks with 2-cell ghosts (the 5^3 filter's
        # radius): outside the step; bytes = one cell read per brick cell
        # written, ghosts included
        B, G = (64, 64, 64), (2, 2, 2)
        nb = vkt.vktBrickDecomposeGetNumBricks(hs, B)
        bricks = []
        for bz in range(nb[2]):
            for by in range(nb[1]):
                for bx in range(nb[0]):
                    dx, dy, dz = vkt.vktBrickDecomposeGetBrickDims(hs, B, G, (bx, by, bz))
                    bricks.append(torch.empty((dz, dy, dx), dtype=src.dtype, device=src.device))
        hb = [vkt.volume_from_tensor(t) for t in bricks]
        handles += hb
        nbc = sum(t.numel() for t in bricks)
        ops.append(dict(case=f"brick_decompose_64_g2_{name}",
                        fn=lambda hb=hb, hs=hs: vkt.vktBrickDecompose(hb, hs, B, G, "clamp"),
                        voxels=n, bytes=2 * nbc * cb, step=False))
    torch.cuda.synchronize()

    def timed(op_list, K, W):
        for _ in range(W):
            for o in op_list:
                o["fn"]()
        torch.cuda.synchronize()
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(2 * len(op_list))]
               for _ in range(K)]
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record(stream)
        for s in range(K):
            for i, o in enumerate(op_list):
                evs[s][2 * i].record(stream)
                o["fn"]()
                evs[s][2 * i + 1].record(stream)
        t1.record(stream)
        torch.cuda.synchronize()
        vkt.vktSynchronize()
        per = [sum(evs[s][2 * i].elapsed_time(evs[s][2 * i + 1]) for s in range(K)) / K
               for i in range(len(op_list))]
        return t0.elapsed_time(t1) / K, per

    step_ops = [o for o in ops if o["step"]]
    print(f"[bench] transforms, warmup {args.warmup}", file=sys.stderr, flush=True)
    ms_step, per = timed(step_ops, args.steps, args.warmup)
    extra = [o for o in ops if not o["step"]]
    _, per_extra = timed(extra, max(1, args.steps // 2), 1)
    per_case = []
    for o, ms in list(zip(step_ops, per)) + list(zip(extra, per_extra)):
        gbs = o["bytes"] / (ms * 1e-3) / 1e9
        per_case.append(dict(case=o["case"], ms=ms, in_step=o["step"],
                             gvoxels_s=o["voxels"] / (ms * 1e-3) / 1e9, hbm_gbs=gbs,
                             hbm_frac=gbs / HBM_PEAK_GBS, algorithmic_bytes=o["bytes"]))
    dom = max((p for p in per_case if p["in_step"]), key=lambda p: p["ms"])
    roof = {"bound": "hbm", "achieved": dom["hbm_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": dom["hbm_frac"], "traffic": stored_traffic(dom["case"], "resample"),
            "kernel_case": dom["case"]}
    voxels = sum(o["voxels"] for o in step_ops)

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        print("[bench] timing the CPU oracle baseline", file=sys.stderr, flush=True)
        t_cpu = 0.0
        for name, src in vols:
            h = src.cpu().numpy()
            Z, Y, X = h.shape
            t0 = time.perf_counter()
            oracle.resample(h, (X // 2, Y // 2, Z // 2))
            oracle.flip(h, int(np.argmax([X, Y, Z])))
            t_cpu += time.perf_counter() - t0
        cpu = {"value": voxels / t_cpu / 1e9, "unit": "Gvoxels/s", "cores": 1, "kind": "oracle",
               "sample": "the oracle's resample (FP64) and flip of both whole 512^3 volumes, "
                         "one thread"}
    line = {
        "metric": "Gvoxels/s Resample(1/2) + Flip(longest axis) on 1 MI355X",
        "value": voxels / (ms_step * 1e-3) / 1e9, "unit": "Gvoxels/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u8+f32", "data": "synthetic",
        "config": {"workload": "transforms",
                   "cases": ["resample 512^3 -> 256^3 and flip along x of the u8 CT-like "
                             "phantom and the f32 smoothed-noise field"]},
        "roofline": roof, "cpu_baseline": cpu, "per_case": per_case,
    }
    for h in handles:
        vkt.vktStructuredVolumeDestroy(h)
    return line


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(a single volume would shard along z with an r-plane halo exchange)",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2203_10213_amd import vkt
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.copy_probe:
        copy_probe()
        return
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.precision is None:
        args.precision = "fp32" if args.workload in ("c1", "c2", "c2a", "c2b") else "auto"
    stream = torch.cuda.current_stream()
    vkt.vktSetStream(stream)
    vkt.vktSetPrecision(args.precision)
    vkt.vktSetSeparable(args.separable)
    vkt.vktSetInt8Matrix(args.int8_matrix)
    if args.workload == "c4":
        print(json.dumps(run_batched(args, vkt, torch)))
        return
    if args.workload == "transforms":
        print(json.dumps(run_transforms(args, vkt, torch)))
        return
    print(f"[bench] building inputs for {args.workload}", file=sys.stderr, flush=True)
    cases = make_cases(args.workload, dev)
    for c in cases:
        c["path"] = kernel_path(c, args.precision, args.separable, args.int8_matrix)
        c["dst"] = torch.empty_like(c["src"])
        c["hs"] = vkt.volume_from_tensor(c["src"])
        c["hd"] = vkt.volume_from_tensor(c["dst"])
        c["hf"] = (vkt.vktFilterCreate(c["w"]) if c["D"] is None
                   else vkt.vktFilterCreateInt(c["w"], c["D"]))
    torch.cuda.synchronize()

    def step(evs=None):
        for i, c in enumerate(cases):
            if evs is not None:
                evs[i][0].record(stream)
            vkt.vktApplyFilter(c["hd"], c["hs"], c["hf"], vkt.vktAddressModeClamp)
            if evs is not None:
                evs[i][1].record(stream)

    print(f"[bench] warmup {args.warmup}", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        step()
    vkt.vktSynchronize()
    torch.cuda.synchronize()

    K = args.steps
    evs = [[[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in cases]
           for _ in range(K)]
    t_begin = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_begin.record(stream)
    for s in range(K):
        step(evs[s])
    t_end.record(stream)
    torch.cuda.synchronize()
    vkt.vktSynchronize()
    total_ms = t_begin.elapsed_time(t_end)
    ms_step = total_ms / K
    voxels = sum(c["voxels"] for c in cases)
    value = voxels / (ms_step * 1e-3) / 1e9

    per_case = []
    for i, c in enumerate(cases):
        ms = sum(evs[s][i][0].elapsed_time(evs[s][i][1]) for s in range(K)) / K
        per_case.append(case_roofline(c, ms))
    dom = max(range(len(cases)), key=lambda i: per_case[i]["ms"])
    d = per_case[dom]
    roof = dict(d["roofline"])
    roof["kernel_case"] = d["case"]
    roof["traffic"] = stored_traffic(d["case"], d["path"])

    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle baseline", file=sys.stderr, flush=True)
        cpu = cpu_baseline(cases, args.cpu_seconds)

    dtype = {torch.uint8: "u8", torch.uint16: "u16", torch.float32: "f32"}
    line = {
        "metric": ("Gvoxels/s ApplyFilter on 1 MI355X" +
                   (" (rank-1 separable fast path)" if args.separable else "")),
        "value": value, "unit": "Gvoxels/s", "n_gpus": 1, "steps": K,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "+".join(sorted({arith_dtype(c, args.precision) for c in cases})),
        "data": "synthetic",
        "config": {"workload": args.workload,
                   "cases": [f"{c['name']} ({dtype[c['src'].dtype]} "
                             f"{'x'.join(str(v) for v in reversed(c['src'].shape))})"
                             for c in cases],
                   "address_mode": "clamp", "precision": args.precision,
                   "separable": bool(args.separable)},
        "roofline": roof,
        "cpu_baseline": cpu,
        "per_case": per_case,
    }
    for c in cases:
        vkt.vktFilterDestroy(c["hf"])
        vkt.vktStructuredVolumeDestroy(c["hs"])
        vkt.vktStructuredVolumeDestroy(c["hd"])
    print(json.dumps(line))


if __name__ == "__main__":
    main()
