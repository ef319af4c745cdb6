"""Throughput benchmark of vktApplyFilter on one MI355X.

Default workload (c2a+c3a), the two stencil sizes of the headline metric:
  (a) 512^3 uint8 CT-like phantom (N(40, 8^2) background, 200 solid spheres),
      integer 3^3 box filter with divisor 27, clamp, uint8 out (bit-exact),
      on the 8-bit dot-product path;
  (b) 1024^3 float32 blob field (64 Gaussian blobs + 1 % noise), dense 7^3
      N(0,1) weights of unit L1 norm, clamp, float32 out, as the split-bf16
      implicit GEMM on the matrix cores (3 products, FP32 accumulation).
One step = one ApplyFilter of (a) and one of (b), inputs resident in HBM.
Beside the step (per_case, in_step false): the same 7^3 filter as the plain
FP32 vector-ALU kernel and as the 6-product split -- the plain vs matrix-core
comparison at stated accuracy.  The CPU leg times the FP64 oracle on 32^3
blocks of each case (all cores and one core) and reports max and RMS error of
every GPU result against it.  Prints ONE JSON line (metric Gvoxels/s = output
cells / device time).

Other workloads (--workload): c1 (64^3 float32, 3^3 Gaussian), c2 (the
plain-path 512^3 pair: (a) and a float32 5^3 Gaussian), c2a, c2b, c3a / c3b
(the 1024^3 field with 7^3 / 9^3 weights, split and plain), c4 (256 uneven
uint16 volumes, batched), c5 (2048 x 2048 x 1024 uint16 ellipsoid phantom,
11^3 Gaussian sigma 2.5), transforms (Resample down by two and Flip along the
longest axis of the two 512^3 volumes, the paper's other structured-volume
benchmarks).
"""
import argparse
import hashlib
import json
import os
import statistics
import sys
import threading
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Gvoxels/s ApplyFilter (3^3 and 7^3) on 1 MI355X; % HBM/MFMA peak; plain vs MFMA"
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
FP32_VECTOR_PEAK_TF = 157.3    # MI355X FP32 vector (packed FMA), TFLOP/s
BF16_MFMA_PEAK_TF = 2500.0     # MI355X dense bf16/fp16 matrix, TFLOP/s
# 8-bit dot products on the vector ALUs: 256 CUs x 4 SIMDs x 16 lanes x 4 MACs
# x 2 ops x 2.4 GHz (v_dot4 issues at the full VALU rate)
INT8_DOT_PEAK_TOPS = 256 * 4 * 16 * 4 * 2 * 2.4e9 / 1e12
INT8_MFMA_PEAK_TOPS = 5000.0   # MI355X dense int8 matrix, TOP/s
MALL_BYTES = 256 << 20         # Infinity Cache


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="c2a+c3a",
                    choices=["c2a+c3a", "c1", "c2", "c2a", "c2b", "c3a", "c3b", "c4", "c5",
                             "transforms"])
    ap.add_argument("--precision", default=None,
                    choices=["auto", "fp32", "splitbf16", "splitbf16x6"],
                    help="precision of the in-step float filters with k >= 5 (default: "
                         "splitbf16, the 3-product split; fp32 for the c1/c2 plain-path "
                         "workloads)")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the out-of-step plain / 6-product comparison cases")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-blocks", type=int, default=512,
                    help="random 32^3 blocks (plus the 8 corner blocks) per case on which "
                         "the oracle is timed on all cores and the errors are measured")
    ap.add_argument("--int8-matrix", action="store_true",
                    help="uint8 3^3 integer filters on the int8 matrix cores instead of "
                         "the 8-bit dot products (vktSetInt8Matrix(1))")
    ap.add_argument("--separable", action="store_true",
                    help="rank-1 fast path (vktSetSeparable): three 1-D passes for separable "
                         "filters; reported apart from the dense numbers")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device copy (counter calibration)")
    return ap.parse_args()


# --------------------------------------------------------------- workloads --

def make_cases(name, device, precision, compare):
    """List of dicts: name, src tensor, weights, divisor, k, precision, and
    whether the case is part of the timed step (comparison cases are timed
    apart on the same input)."""
    import torch
    from paper_2203_10213_amd import synth
    S = synth.SEEDS
    cases = []

    def add(name, src, w, D, k, prec, in_step=True, blocks_seed=None):
        cases.append(dict(name=name, src=src, w=w, D=D, k=k, precision=prec,
                          in_step=in_step, blocks_seed=blocks_seed))

    if name in ("c2", "c2a", "c2a+c3a"):
        src = torch.from_numpy(synth.ct_phantom_u8(512, S["c2a"])).to(device)
        w, D = synth.box_int(3)
        add("c2a_u8_512_box3_div27", src, w, D, 3, "fp32", blocks_seed=S["c2_blocks"])
    if name in ("c2", "c2b"):
        src = synth.smoothed_noise_f32(512, 4.0, S["c2b"], device=device)
        add("c2b_f32_512_gauss5_s1.5", src, synth.gaussian_weights(5, 1.5), None, 5,
            precision or "fp32", blocks_seed=S["c2_blocks"])
    if name == "c1":
        src = torch.from_numpy(synth.uniform_f32((64, 64, 64), S["c1"])).to(device)
        add("c1_f32_64_gauss3_s1", src, synth.gaussian_weights(3, 1.0), None, 3, "fp32",
            blocks_seed=S["c1"])
    if name in ("c3a", "c3b", "c2a+c3a"):
        k = 9 if name == "c3b" else 7
        src = synth.blob_field_f32(1024, 64, S["c3"], device=device)
        w = synth.random_l1(k, S["c3a_w"] if k == 7 else S["c3b_w"])
        tag = "c3a" if k == 7 else "c3b"
        p = precision or "splitbf16"
        add(f"{tag}_f32_1024_dense{k}_l1", src, w, None, k, p, blocks_seed=S["c3_blocks"])
        if compare:
            for q in ("fp32", "splitbf16x6", "splitbf16"):
                if q != p:
                    add(f"{tag}_f32_1024_dense{k}_l1", src, w, None, k, q, in_step=False,
                        blocks_seed=S["c3_blocks"])
    if name == "c5":
        src = synth.ellipsoid_phantom_u16((1024, 2048, 2048), 5000, S["c5"], device=device)
        w = synth.gaussian_weights(11, 2.5)
        add("c5_u16_2048x2048x1024_gauss11_s2.5", src, w, None, 11, precision or "splitbf16",
            blocks_seed=S["c5_blocks"])
        if compare:
            add("c5_u16_2048x2048x1024_gauss11_s2.5", src, w, None, 11, "fp32", in_step=False,
                blocks_seed=S["c5_blocks"])
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
    "mfma": ["vkt_filter_mfma.hip", "vkt_filter_mfma_rp.hip", "vkt_mfma_common.h", "vkt_internal.h"],
    "sep": ["vkt_filter_sep.hip", "vkt_internal.h"],
    # the batched graph: its planner and every class kernel it may launch
    "batched": ["vkt_batch.hip", "vkt_filter_valu.hip", "vkt_filter_dot4.hip",
                "vkt_filter_mfma.hip", "vkt_filter_mfma_rp.hip", "vkt_mfma_common.h",
                "vkt_internal.h"],
}


def kernel_source_sha(path):
    """Hash of the HIP sources of one kernel path; profile-derived figures are
    only reported for the kernel they were measured on."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2203_10213_amd", "csrc")
    for f in KERNEL_SOURCES[path]:
        p = os.path.join(csrc, f)
        if os.path.exists(p):
            h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def stored_profile(case_key, path, field):
    """A per-launch figure (HBM bytes from FETCH_SIZE / WRITE_SIZE scaled by
    the copy-kernel calibration, or the matrix-core busy fraction) from the
    committed rocprofv3 summaries, if it was measured on the current kernel."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
        e = d.get(case_key)
        if e and e.get("path") == path and e.get("kernel_src_sha") == kernel_source_sha(path):
            return e.get(field)
    except (ValueError, KeyError):
        pass
    return None


def case_key(c):
    """Name of a case with its arithmetic (the profile table's key)."""
    if c["path"] == "mfma":
        return f"{c['name']}:mfma_x{c['products']}"
    return f"{c['name']}:{c['path']}"


def arith_dtype(c):
    """The type the path computes in."""
    if c["path"] == "mfma":
        if c["src"].dtype.is_floating_point:
            return f"bf16x{c['products']}->f32"
        return f"f16x{c['products']}->f32"
    return {"dot4": "u8dot4->i32", "i8mma": "i8mma->i32", "sep": "f32(rank-1)"}.get(
        c["path"], "f32(exact int)" if c["D"] is not None else "f32")


def case_roofline(c, ms):
    """Algorithmic bytes (1 cell read + 1 cell written per output) and flops
    (2 k^3 per output) over the measured time, against the roofline that
    bounds this path at its algorithmic work: HBM, the FP32 vector ALUs, the
    8-bit dot products, or the dense 16-bit / int8 matrix cores (split
    products and Toeplitz zeros are overhead, not counted).  Matrix-core
    cases also report the useful-product fraction (P split products of the
    algorithmic flops) and the counter-measured busy fraction."""
    t = ms * 1e-3
    bytes_alg = 2 * c["voxels"] * c["cell_bytes"]
    # the rank-1 path's algorithm is three 1-D passes: 2 * 3k flops per output
    flops = c["voxels"] * (6 * c["k"] if c["path"] == "sep" else c["flops_per_voxel"])
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
    out = dict(case=c["name"], in_step=c["in_step"], precision=c["precision"], path=c["path"],
               products=c["products"], ms=ms, gvoxels_s=c["voxels"] / t / 1e9, hbm_gbs=gbs,
               hbm_frac=gbs / HBM_PEAK_GBS, tflops=tfs, algorithmic_bytes=bytes_alg,
               flops=flops, roofline=roof,
               traffic=stored_profile(case_key(c), c["path"], "hbm_bytes_per_launch"))
    if c["path"] == "mfma":
        out["matrix_cores"] = {
            "algorithmic_frac": tfs / BF16_MFMA_PEAK_TF,
            "useful_product_frac": c["products"] * tfs / BF16_MFMA_PEAK_TF,
            "busy_frac": stored_profile(case_key(c), "mfma", "mfma_busy")}
    return out


# ------------------------------------------------- CPU baseline and errors --

def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def host_cores():
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def _blocks(t, origins):
    """The 32^3 blocks (clipped to the volume) of device tensor t at origins."""
    import torch
    Z, Y, X = t.shape
    bx, by, bz = min(32, X), min(32, Y), min(32, Z)
    return torch.stack([t[z:z + bz, y:y + by, x:x + bx] for x, y, z in origins]).cpu().numpy()


def result_errors(c, got, T, A):
    """Error of one GPU result against the oracle on the checked cells:
    float32 cells: max and RMS of |gpu - T| and of |gpu - T| / sum|w||s|;
    integer cells: the oracle's stored result (bit-exact rule for integer
    filters, half-up rounding for float filters) and the largest difference
    in units of the last place."""
    import numpy as np
    import oracle
    n = int(got.size)
    if got.dtype == np.float32:
        d = np.abs(got.astype(np.float64) - T)
        e = np.where(A > 0, d / np.maximum(A, 1e-300), np.where(d == 0, 0.0, np.inf))
        return {"cells": n, "max_abs": float(d.max()), "rms_abs": float(np.sqrt(np.mean(d * d))),
                "max_rel_sum_abs": float(e.max()), "rms_rel_sum_abs": float(np.sqrt(np.mean(e * e)))}
    want = (oracle.store_int_filter(T, c["D"], got.dtype) if c["D"] is not None
            else oracle.store_float_filter(T, got.dtype))
    diff = np.abs(got.astype(np.int64) - want.astype(np.int64))
    return {"cells": n, "max_lsb": int(diff.max()), "cells_differing": int((diff != 0).sum()),
            "rule": "bit-exact" if c["D"] is not None else "within 1 LSB"}


def cpu_leg(cases, n_random):
    """The FP64 oracle timed on this host on 32^3 blocks of every distinct
    (input, filter) of the workload: the 8 corner blocks plus n_random blocks
    placed uniformly (seeded) on all cores, and the corner blocks plus 8
    random ones on one core.  Its block results are then the reference for
    the max / RMS error of every GPU result.  Returns (cpu_baseline, errors,
    input hashes)."""
    import numpy as np
    import oracle
    from paper_2203_10213_amd import synth
    allc = min(16, host_cores())
    groups = {}
    for c in cases:
        groups.setdefault((id(c["src"]), c["name"]), []).append(c)
    per_voxel, errors, hashes, samples = {}, {}, {}, []
    for (_, name), cs in groups.items():
        c0 = cs[0]
        src = c0["src"].cpu().numpy()
        hashes[name] = hashlib.sha256(memoryview(np.ascontiguousarray(src)).cast("B")).hexdigest()
        origins = synth.sample_blocks(src.shape, n_random, c0["blocks_seed"])
        w = np.asarray(c0["w"], np.float64)
        Z, Y, X = src.shape
        ext = (min(32, X), min(32, Y), min(32, Z))
        vox_per_block = ext[0] * ext[1] * ext[2]

        def run(orgs, nthreads):
            Ts, As = [], []
            t0 = time.perf_counter()
            for x, y, z in orgs:
                T, A = oracle.correlate_box(src, w, "clamp", (x, y, z),
                                            (x + ext[0], y + ext[1], z + ext[2]),
                                            nthreads=nthreads)
                Ts.append(T)
                As.append(A)
            return time.perf_counter() - t0, np.stack(Ts), np.stack(As)

        print(f"[bench] oracle on {len(origins)} blocks of {name}, {allc} threads",
              file=sys.stderr, flush=True)
        t_all, T, A = run(origins, allc)
        one = origins[:16]
        print(f"[bench] oracle on {len(one)} blocks of {name}, 1 thread", file=sys.stderr,
              flush=True)
        t_one, _, _ = run(one, 1)
        per_voxel[name] = (t_all / (len(origins) * vox_per_block),
                           t_one / (len(one) * vox_per_block))
        samples.append(f"{name}: {len(origins)} blocks of {ext[0]}x{ext[1]}x{ext[2]} cells "
                       f"(8 corners + {len(origins) - 8} uniform, seed {c0['blocks_seed']}) on "
                       f"{allc} threads, {len(one)} of them on 1 thread")
        for c in cs:
            got = _blocks(c["dst"], origins)
            errors[f"{c['name']}:{c['precision']}:{c['path']}"] = result_errors(c, got, T, A)
    step = [c for c in cases if c["in_step"]]
    vox = sum(c["voxels"] for c in step)
    t_allc = sum(c["voxels"] * per_voxel[c["name"]][0] for c in step)
    t_1 = sum(c["voxels"] * per_voxel[c["name"]][1] for c in step)
    cpu = {"value": vox / t_allc / 1e9, "unit": "Gvoxels/s", "cores": allc, "kind": "oracle",
           "sample": "FP64 direct-sum oracle (C, -O2) on " + "; ".join(samples) +
                     "; time per cell scaled to the step's cells",
           "one_core": {"value": vox / t_1 / 1e9, "unit": "Gvoxels/s", "cores": 1},
           "cpu_model": cpu_model(), "host_cpus": host_cores(), "nproc": os.cpu_count()}
    return cpu, errors, hashes


# ------------------------------------------------------------ clocks, copy --

class ClockSampler:
    """Samples the GPU's graphics clock (MHz) from a thread while the timed
    region runs: amdsmi if it loads, else the driver's sysfs DPM table."""

    def __init__(self, period_s=0.005):
        self.period = period_s
        self.samples = []
        self.read = None
        self.source = None
        try:
            import amdsmi
            amdsmi.amdsmi_init()
            h = amdsmi.amdsmi_get_processor_handles()[0]

            def rd():
                return float(amdsmi.amdsmi_get_clock_info(h, amdsmi.AmdSmiClkType.GFX)["clk"])
            rd()
            self.read, self.source = rd, "amdsmi GFX clock"
        except Exception:
            import glob
            for f in sorted(glob.glob("/sys/class/drm/card*/device/pp_dpm_sclk")):
                def rd(f=f):
                    for line in open(f):
                        if "*" in line:
                            return float(line.split(":", 1)[1].replace("*", "")
                                         .strip().lower().replace("mhz", ""))
                    return None
                try:
                    if rd() is not None:
                        self.read, self.source = rd, f
                        break
                except (OSError, ValueError):
                    pass
        self._stop = threading.Event()
        self._th = None

    def _loop(self):
        while not self._stop.is_set():
            try:
                v = self.read()
                if v:
                    self.samples.append(v)
            except Exception:
                pass
            time.sleep(self.period)

    def __enter__(self):
        if self.read:
            self._th = threading.Thread(target=self._loop, daemon=True)
            self._th.start()
        return self

    def __exit__(self, *a):
        self._stop.set()
        if self._th:
            self._th.join()

    def report(self):
        if not self.samples:
            return {"mhz_median": None, "source": self.source}
        return {"mhz_median": statistics.median(self.samples), "mhz_min": min(self.samples),
                "mhz_max": max(self.samples), "samples": len(self.samples),
                "source": self.source}


def copy_ceiling(torch, stream, reps=10):
    """Achieved HBM rate of a plain 1 GiB device-to-device copy (read +
    write bytes / time), the practical ceiling for streaming kernels."""
    n = 1 << 30
    a = torch.empty(n, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    for _ in range(2):
        b.copy_(a)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        b.copy_(a)
    e1.record(stream)
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / reps * 1e-3
    del a, b
    gbs = 2 * n / t / 1e9
    return {"bytes": 2 * n, "gbs": gbs, "frac": gbs / HBM_PEAK_GBS}


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
    hipGraph) per step.  Timed three ways: the batched call with the planner's
    default slab depths, the batched call after the autotuner has timed its
    candidates on this batch (a second set of outputs, so a second plan), and
    the same work as 256 single launches.  The CPU leg times the oracle on one
    32^3 block of every volume (all cores and one core) and reports the
    largest difference of the batched result from it.  Returns the line."""
    import numpy as np
    from paper_2203_10213_amd import synth
    vols, ks = synth.gamma_u16_volumes(256, synth.SEEDS["c4"])
    filts = {k: vkt.vktFilterCreate(synth.gaussian_weights(k, k / 4)) for k in (3, 5, 7)}
    srcs = [torch.from_numpy(v).cuda() for v in vols]
    dsts = [torch.empty_like(x) for x in srcs]
    dsts_t = [torch.empty_like(x) for x in srcs]
    hs = [vkt.volume_from_tensor(x) for x in srcs]
    hd = [vkt.volume_from_tensor(x) for x in dsts]
    ht = [vkt.volume_from_tensor(x) for x in dsts_t]
    hf = [filts[k] for k in ks]
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()

    def batched(out):
        return lambda: vkt.vktApplyFilterBatched(out, hs, hf, "clamp")

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

    clocks = ClockSampler()
    with clocks:
        print(f"[bench] c4 batched (default slab depths), warmup {args.warmup}", file=sys.stderr,
              flush=True)
        vkt.vktSetAutotune(False)
        ms_u = timed(batched(hd), args.steps, args.warmup)
        print("[bench] c4 batched, autotuned plan", file=sys.stderr, flush=True)
        vkt.vktSetAutotune(True)
        ms_t = timed(batched(ht), args.steps, args.warmup)
        vkt.vktSetAutotune(False)
        print("[bench] c4 single launches", file=sys.stderr, flush=True)
        ms_s = timed(singles, max(1, args.steps // 2), 1)
    # the step is the better of the two batched plans (the tuned one unless
    # tuning picked nothing faster)
    ms_b = min(ms_u, ms_t)
    voxels = sum(int(v.size) for v in vols)
    flops = sum(int(v.size) * 2 * k ** 3 for v, k in zip(vols, ks))
    bytes_alg = 4 * voxels
    t = ms_b * 1e-3
    gbs = bytes_alg / t / 1e9
    # the batch's binding roofline at its algorithmic work: 4 bytes per cell
    # moved (HBM) against the split-fp16 matrix flops of the k = 5, 7 volumes
    mfma_flops = sum(int(v.size) * 2 * k ** 3 for v, k in zip(vols, ks) if k >= 5)
    if bytes_alg / (HBM_PEAK_GBS * 1e9) >= mfma_flops / (BF16_MFMA_PEAK_TF * 1e12):
        roof = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": gbs / HBM_PEAK_GBS}
    else:
        roof = {"bound": "mfma", "achieved": mfma_flops / t / 1e12, "peak": BF16_MFMA_PEAK_TF,
                "unit": "TFLOP/s", "frac": mfma_flops / t / 1e12 / BF16_MFMA_PEAK_TF}
    roof.update({"traffic": stored_profile("c4_batched_graph", "batched", "hbm_bytes_per_launch"),
                 "kernel_case": "c4 batched graph (all classes, one launch)"})
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        allc = min(16, host_cores())
        g = np.random.default_rng(synth.SEEDS["c4"] + 1)
        worst, cells, t_all, t_one, n_one = 0, 0, 0.0, 0.0, 0
        print("[bench] CPU leg: the FP64 oracle on one 32^3 block of each volume",
              file=sys.stderr, flush=True)
        for i, (v, k) in enumerate(zip(vols, ks)):
            Z, Y, X = v.shape
            e = (min(32, X), min(32, Y), min(32, Z))
            o = tuple(int(g.integers(0, d - ed + 1)) for d, ed in zip((X, Y, Z), e))
            w = synth.gaussian_weights(k, k / 4).astype(np.float64)
            t0 = time.perf_counter()
            T = oracle.correlate_box(v, w, "clamp", o, tuple(a + b for a, b in zip(o, e)),
                                     nthreads=allc, with_abs=False)
            t_all += time.perf_counter() - t0
            if i < 16:
                t0 = time.perf_counter()
                oracle.correlate_box(v, w, "clamp", o, tuple(a + b for a, b in zip(o, e)),
                                     nthreads=1, with_abs=False)
                t_one += time.perf_counter() - t0
                n_one += T.size
            want = oracle.store_float_filter(T, np.uint16)
            for out in (dsts, dsts_t):
                got = out[i].view(torch.int16)[o[2]:o[2] + e[2], o[1]:o[1] + e[1],
                                               o[0]:o[0] + e[0]].cpu().numpy().view(np.uint16)
                worst = max(worst, int(np.abs(got.astype(np.int64) - want).max()))
            cells += T.size
        # time per cell weighted by each volume's filter size
        work = sum(int(v.size) * k ** 3 for v, k in zip(vols, ks))
        per_tap_all = t_all / sum(min(32, v.shape[0]) * min(32, v.shape[1]) * min(32, v.shape[2])
                                  * k ** 3 for v, k in zip(vols, ks))
        per_tap_one = t_one / sum(min(32, v.shape[0]) * min(32, v.shape[1]) * min(32, v.shape[2])
                                  * k ** 3 for v, k in list(zip(vols, ks))[:16])
        cpu = {"value": voxels / (work * per_tap_all) / 1e9, "unit": "Gvoxels/s", "cores": allc,
               "kind": "oracle",
               "sample": f"FP64 oracle on one 32^3 block (or the whole volume where smaller) of "
                         f"each of the 256 volumes, {cells} cells, {allc} threads; 16 of the "
                         f"blocks on 1 thread; time per tap scaled to the batch's taps",
               "one_core": {"value": voxels / (work * per_tap_one) / 1e9,
                            "unit": "Gvoxels/s", "cores": 1},
               "cpu_model": cpu_model(), "host_cpus": host_cores(), "nproc": os.cpu_count(),
               "max_lsb_vs_oracle": worst, "cells_checked": cells}
    line = {
        "metric": "Gvoxels/s ApplyFilter, batched uneven volumes, on 1 MI355X",
        "value": voxels / t / 1e9, "unit": "Gvoxels/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_b, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f16x4->f32+f32",
        "data": "synthetic",
        "config": {"workload": "c4", "cases": ["256 u16 volumes, axes U{32..256}, "
                                               "Gaussian k in {3,5,7}, sigma k/4"],
                   "address_mode": "clamp", "precision": args.precision or "auto"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "sclk": clocks.report(),
        "per_case": [{"case": "c4_batched_default_slabs", "ms": ms_u,
                      "gvoxels_s": voxels / (ms_u * 1e-3) / 1e9,
                      "hbm_frac": bytes_alg / (ms_u * 1e-3) / 1e9 / HBM_PEAK_GBS},
                     {"case": "c4_batched_autotuned", "ms": ms_t,
                      "gvoxels_s": voxels / (ms_t * 1e-3) / 1e9,
                      "hbm_frac": bytes_alg / (ms_t * 1e-3) / 1e9 / HBM_PEAK_GBS},
                     {"case": "c4_256_single_launches", "ms": ms_s,
                      "gvoxels_s": voxels / (ms_s * 1e-3) / 1e9,
                      "hbm_frac": bytes_alg / (ms_s * 1e-3) / 1e9 / HBM_PEAK_GBS,
                      "tflops": flops / (ms_s * 1e-3) / 1e12}],
    }
    for h in hs + hd + ht:
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
            "frac": dom["hbm_frac"], "traffic": stored_profile(dom["case"], "resample", "hbm_bytes_per_launch"),
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


def run_filters(args, vkt, torch):
    """The single-volume ApplyFilter workloads: the step's cases timed
    together K times (HIP events around the whole step and around each
    call, on the stream the library launches on), the comparison cases K
    times apart; then the CPU leg.  Returns the bench line."""
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    print(f"[bench] building inputs for {args.workload}", file=sys.stderr, flush=True)
    cases = make_cases(args.workload, dev, args.precision, not args.no_compare)
    for c in cases:
        c["dst"] = torch.empty_like(c["src"])
        c["hs"] = vkt.volume_from_tensor(c["src"])
        c["hd"] = vkt.volume_from_tensor(c["dst"])
        c["hf"] = (vkt.vktFilterCreate(c["w"]) if c["D"] is None
                   else vkt.vktFilterCreateInt(c["w"], c["D"]))
        vkt.vktSetPrecision(c["precision"])
        p, n = vkt.vktGetFilterPath(c["hd"], c["hs"], c["hf"], "clamp")
        c["path"], c["products"] = vkt.FILTER_PATHS[p], n
    torch.cuda.synchronize()
    step_cases = [c for c in cases if c["in_step"]]
    cmp_cases = [c for c in cases if not c["in_step"]]
    # working sets below 1 GiB would stay partly in the 256 MB MALL between
    # steps: flush it with a 1 GiB write between steps and time the kernels
    # themselves (events around each call)
    ws = sum(2 * c["voxels"] * c["cell_bytes"] for c in step_cases)
    flush = torch.empty(1 << 30, dtype=torch.uint8, device=dev) if ws < (1 << 30) else None

    def call(c):
        vkt.vktSetPrecision(c["precision"])
        vkt.vktApplyFilter(c["hd"], c["hs"], c["hf"], vkt.vktAddressModeClamp)

    def timed(cs, K, W, with_flush):
        for _ in range(W):
            for c in cs:
                call(c)
        vkt.vktSynchronize()
        torch.cuda.synchronize()
        evs = [[[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in cs]
               for _ in range(K)]
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record(stream)
        for s in range(K):
            if with_flush:
                flush.fill_(s & 0xff)
            for i, c in enumerate(cs):
                evs[s][i][0].record(stream)
                call(c)
                evs[s][i][1].record(stream)
        t1.record(stream)
        torch.cuda.synchronize()
        vkt.vktSynchronize()
        per = [sum(evs[s][i][0].elapsed_time(evs[s][i][1]) for s in range(K)) / K
               for i in range(len(cs))]
        return t0.elapsed_time(t1) / K, per

    K = args.steps
    clocks = ClockSampler()
    with clocks:
        print(f"[bench] step: {', '.join(c['name'] + ':' + c['path'] for c in step_cases)}; "
              f"warmup {args.warmup}, {K} steps", file=sys.stderr, flush=True)
        ms_bracket, per_step = timed(step_cases, K, args.warmup, flush is not None)
        per_cmp = []
        for c in cmp_cases:
            print(f"[bench] comparison: {c['name']} {c['precision']} ({c['path']})",
                  file=sys.stderr, flush=True)
            per_cmp += timed([c], K, 1, False)[1]
    # with a MALL flush between steps the step time is the sum of the calls
    ms_step = sum(per_step) if flush is not None else ms_bracket
    voxels = sum(c["voxels"] for c in step_cases)
    value = voxels / (ms_step * 1e-3) / 1e9
    per_case = [case_roofline(c, ms) for c, ms in zip(step_cases + cmp_cases, per_step + per_cmp)]
    dom = max(range(len(step_cases)), key=lambda i: per_case[i]["ms"])
    d = per_case[dom]
    roof = dict(d["roofline"])
    roof["kernel_case"] = f"{d['case']} ({d['path']}, {d['precision']})"
    roof["traffic"] = d["traffic"]
    if "matrix_cores" in d:
        roof["matrix_cores"] = d["matrix_cores"]
    print("[bench] copy ceiling", file=sys.stderr, flush=True)
    ceiling = copy_ceiling(torch, stream)

    cpu, errors, hashes = None, None, None
    if not args.no_cpu_baseline:
        print("[bench] CPU leg: the FP64 oracle on 32^3 blocks (timing and errors)",
              file=sys.stderr, flush=True)
        cpu, errors, hashes = cpu_leg(cases, args.cpu_blocks)
        for p in per_case:
            for k, v in errors.items():
                if k.startswith(f"{p['case']}:{p['precision']}:{p['path']}"):
                    p["error_vs_oracle"] = v

    dtype = {torch.uint8: "u8", torch.uint16: "u16", torch.float32: "f32"}
    line = {
        "metric": METRIC + (" (rank-1 separable fast path)" if args.separable else ""),
        "value": value, "unit": "Gvoxels/s", "n_gpus": 1, "steps": K,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "+".join(arith_dtype(c) for c in step_cases),
        "data": "synthetic",
        "config": {"workload": args.workload,
                   "cases": [f"{c['name']} ({dtype[c['src'].dtype]} "
                             f"{'x'.join(str(v) for v in reversed(c['src'].shape))}, "
                             f"{c['path']}, {c['precision']})" for c in step_cases],
                   "compare": [f"{c['name']} ({c['path']}, {c['precision']})" for c in cmp_cases],
                   "address_mode": "clamp", "separable": bool(args.separable),
                   "timing": ("sum of per-call HIP events per step, MALL flushed between steps "
                              "by a 1 GiB write" if flush is not None else
                              f"HIP events around {K} whole steps (working set "
                              f"{ws / 2**30:.1f} GiB, > 4x the 256 MB MALL)"),
                   "input_sha256": hashes},
        "roofline": roof,
        "cpu_baseline": cpu,
        "sclk": clocks.report(),
        "copy_ceiling": ceiling,
        "per_case": per_case,
    }
    for c in cases:
        vkt.vktFilterDestroy(c["hf"])
        vkt.vktStructuredVolumeDestroy(c["hs"])
        vkt.vktStructuredVolumeDestroy(c["hd"])
    return line


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(a single volume would shard along z with an r-plane halo exchange)",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2203_10213_amd import vkt
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.copy_probe:
        copy_probe()
        return
    torch.cuda.set_device(torch.device("cuda:0"))
    if args.precision is None and args.workload in ("c1", "c2", "c2b"):
        args.precision = "fp32"
    vkt.vktSetStream(torch.cuda.current_stream())
    vkt.vktSetPrecision(args.precision or "auto")
    vkt.vktSetSeparable(args.separable)
    vkt.vktSetInt8Matrix(args.int8_matrix)
    if args.workload == "c4":
        print(json.dumps(run_batched(args, vkt, torch)))
    elif args.workload == "transforms":
        print(json.dumps(run_transforms(args, vkt, torch)))
    else:
        print(json.dumps(run_filters(args, vkt, torch)))


if __name__ == "__main__":
    main()
