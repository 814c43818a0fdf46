"""Benchmark of the RL-JSDE hot path on one MI355X.

Default workload (``--workload batch64``): 64 synthetic grey images of uneven
size (256x256, 640x480, 1024x768, 1920x1080 or 2048x1536; sinusoids + polygons
on a 128 base), each three-quarter-sampled through its own random recurrent
opaque-quadrant tile of period 2, 4 or 8 sensor pixels; window 32, block 4,
100 iterations, rho 0.7, gamma 0.5. A step is one reconstruction of the whole
batch by the FP32 batched path: one persistent launch replayed from its HIP
graph, reading the float64 measurements. The plain FP64 GPU path (one launch
per image) is timed on the same input beside it, and the FP64 CPU oracle on a
bounded sample of windows drawn across all images.

Other workloads (``--workload``): frame512 (one 512x512 frame, 4x4-sensor
tile, 100 iterations), frame2048 (2048x2048 + N(0, 2^2) noise, 8x8-sensor
tile, 250 iterations), frame8192 (8192x8192 float32 image, 16x16-sensor tile,
250 iterations; FP32 and FP64 read the float32 measurements), paper1200
(1200x1200, 16x16-sensor tile, 100 iterations), quarter512 (the 512x512 frame
under quarter sampling: one transparent quadrant per pixel), dense512 (the
512x512 frame on the dense form: per-class C in device memory, FP64) and
weights512 (a 512x512 frame under a recurrent 4x4 general layout of per-pixel
quadrant weights, dense form, FP64), ljsde64 (a 64x64 frame with a
non-recurrent pattern, plain L-JSDE in FP64: the paper's baseline method) and
ljsde256 / ljsde512 (256x256 / 512x512 frames with a recurrent 4x4-sensor
pattern) and ljsde1200 (the paper's 1200x1200 shape with its 32-pixel period,
the comparison of its Table II), plain L-JSDE, each timed beside the recurrent
FP64 and FP32 batched paths on the same input.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from synth import batch_cases, make_case, random_weights, sense_weights, synthetic_image  # noqa: E402

METRIC = "reconstructed MP/s (FP32 batched vs FP64 plain, same GPU) at \u22640.01 dB PSNR delta"
W, B, RHO, GAMMA = 32, 4, 0.7, 0.5
FP64_TOL = 1e-9                   # FP64 against the oracle: max-abs
FP32_TOL, PSNR_TOL = 0.05, 0.01   # FP32 against the oracle: max-abs (grey levels), PSNR delta (dB)
FLOPS_PER_FREQ_ITER = 30          # factorised form: projection 18, metric 4, update 8
DENSE_FLOPS_PER_FREQ_ITER = 12    # dense form: metric 4, update 8 (eq. (17): one complex multiply-add)
PEAK_FP64_VALU = 78.6e12          # MI355X FP64 vector peak, FLOP/s
PEAK_FP32_VALU = 157.3e12         # MI355X FP32 vector peak (packed), FLOP/s
PEAK_LDS = 128 * 256 * 2.4e9      # LDS bytes/s taken as 128 B/clk per CU, 256 CUs at 2.4 GHz
# LDS reads of the FP32 kernel per window-iteration: each of 64 lanes reads, for
# its 4 positions, the shifted spectra of 4 orientations (16 B each) and its
# q/D and twiddles (2 x 16 B)
LDS_BYTES_PER_WIN_ITER = 64 * 4 * (4 * 16 + 2 * 16)
KERNEL_SOURCES = ["paper_2205_02646_amd/csrc/ljsde_mixed.hip", "paper_2205_02646_amd/csrc/ljsde_device.h",
                  "paper_2205_02646_amd/csrc/ljsde_internal.h"]

WORKLOADS = {
    "frame512": dict(kind="frame", rows=512, cols=512, period=4, iters=100, noise=0.0,
                     desc="512x512 frame, recurrent 4x4-sensor pattern"),
    "frame2048": dict(kind="frame", rows=2048, cols=2048, period=8, iters=250, noise=2.0,
                      desc="2048x2048 frame + N(0,2^2) noise, recurrent 8x8-sensor pattern"),
    "frame8192": dict(kind="frame", rows=8192, cols=8192, period=16, iters=250, noise=0.0, y32=True,
                      desc="8192x8192 float32 frame, recurrent 16x16-sensor pattern (64 interior / 256 classes)"),
    "paper1200": dict(kind="frame", rows=1200, cols=1200, period=16, iters=100, noise=0.0,
                      desc="1200x1200 frame, recurrent 16x16-sensor pattern (period 32 px)"),
    "batch64": dict(kind="batch", n=64, iters=100,
                    desc="64 images of uneven size, own patterns of period 2/4/8"),
    "quarter512": dict(kind="frame", rows=512, cols=512, period=4, iters=100, noise=0.0, shape=0x1,
                       desc="512x512 frame, quarter sampling (one transparent quadrant per pixel), "
                            "recurrent 4x4-sensor pattern"),
    "dense512": dict(kind="frame", rows=512, cols=512, period=4, iters=100, noise=0.0, path="fp64_dense",
                     desc="512x512 frame, recurrent 4x4-sensor pattern, FP64 dense form (per-class C of "
                          "eq. (14) in device memory)"),
    "weights512": dict(kind="weights", rows=512, cols=512, period=4, iters=100, noise=0.0, path="fp64_dense",
                       desc="512x512 frame, general layout (random per-pixel quadrant weights, recurrent "
                            "4x4-sensor tile), FP64 dense form"),
}
WORKLOADS.update({
    "ljsde64": dict(kind="frame", rows=64, cols=64, period=None, iters=100, noise=0.0, path="plain_l",
                    desc="64x64 frame, non-recurrent pattern (every window its own local measurement matrix), "
                         "plain L-JSDE FP64"),
    "ljsde256": dict(kind="frame", rows=256, cols=256, period=4, iters=100, noise=0.0, path="plain_l",
                     desc="256x256 frame, recurrent 4x4-sensor pattern, plain L-JSDE FP64"),
    "ljsde512": dict(kind="frame", rows=512, cols=512, period=4, iters=100, noise=0.0, path="plain_l",
                     desc="512x512 frame, recurrent 4x4-sensor pattern, plain L-JSDE FP64"),
    "ljsde1200": dict(kind="frame", rows=1200, cols=1200, period=16, iters=100, noise=0.0, path="plain_l",
                      desc="1200x1200 frame, recurrent 16x16-sensor pattern (period 32 px), plain L-JSDE FP64"),
})
PEAK_FP64_MFMA = 78.6e12          # MI355X FP64 matrix peak, FLOP/s
HBM_PEAK_GBPS = 8000.0            # MI355X HBM3E
DENSE_KERNEL_SOURCES = ["paper_2205_02646_amd/csrc/ljsde_dense.hip", "paper_2205_02646_amd/csrc/ljsde_window.h",
                        "paper_2205_02646_amd/csrc/ljsde_device.h", "paper_2205_02646_amd/csrc/ljsde_internal.h"]


def _code_only(text: str) -> str:
    """Source text without comments and blank space, so that the hash follows
    the code the counters were taken on, not its comments."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_hash(sources=None) -> str:
    h = hashlib.sha256()
    for f in (sources or KERNEL_SOURCES):
        with open(os.path.join(ROOT, f)) as fh:
            h.update(_code_only(fh.read()).encode())
    return h.hexdigest()[:16]


def load_traffic(workload: str, sources=None):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "kernel_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh).get(workload)
    if not rec or rec.get("kernel_hash") != kernel_hash(sources):
        return None
    return rec.get("hbm_bytes_per_launch")


_ORACLE_IMAGES = []  # (y, tile, shape, weights) per image, inherited by the forked oracle workers


def _oracle_worker(args):
    k, blocks, iters, form = args
    y, tile, shape, weights = _ORACLE_IMAGES[k]
    from oracle import ljsde_oracle as O
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except Exception:  # pragma: no cover
        pass
    out, tr = O.reconstruct(y, tile, W=W, B=B, iters=iters, rho=RHO, gamma=GAMMA, form=form, blocks=blocks,
                            shape=shape, weights=weights, traces=True)
    return [(k, bi, bj, out[B * bi:B * bi + B, B * bj:B * bj + B], tr[(bi, bj)].picks, tr[(bi, bj)].gap)
            for bi, bj in blocks]


def _canon(k: int) -> int:
    # a frequency and its conjugate partner (-sigma, -rho) give the same real output
    s, r = divmod(int(k), W)
    return min(s * W + r, ((-s) % W) * W + (-r) % W)


def divergence(sel_of, picks: dict, gaps: dict) -> dict:
    """Windows whose GPU selection sequence differs from the oracle's: the raw
    count, the count modulo conjugate partners, and the oracle's relative top-2
    metric gap at the first divergence of each (small gaps: near ties)."""
    raw, canon, first = 0, 0, []
    for key, pk in picks.items():
        s = [int(v) for v in sel_of(key)][:len(pk)]
        pk = [int(v) for v in pk]
        if s == pk:
            continue
        raw += 1
        f = next((n for n, (a, b) in enumerate(zip(s, pk)) if a != b), min(len(s), len(pk)) - 1)
        first.append(float(gaps[key][f]))
        canon += [_canon(k) for k in s] != [_canon(k) for k in pk]
    gap = {"min": min(first), "median": float(np.median(first)), "max": max(first)} if first else None
    return {"diverged": raw, "diverged_modulo_conjugation": canon, "oracle_top2_gap_at_first_divergence": gap}


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _run_oracle(tasks, procs):
    import multiprocessing as mp
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(procs) as pool:
        parts = pool.map(_oracle_worker, tasks, chunksize=1)
    return [r for part in parts for r in part], time.perf_counter() - t0


def cpu_baseline(images, iters: int, n_windows: int, seed: int = 1, label: str = ""):
    """Time the FP64 oracle (RL-JSDE form) on a random sample of windows spread
    evenly over the images, over the host cores. ``images``: list of (y, tile,
    shape, weights). Returns (record, {(image, bi, bj): output block},
    {key: selections}, {key: relative top-2 gaps})."""
    rng = np.random.default_rng(seed)
    per = max(1, n_windows // len(images))
    by_image = []
    for y, _, _, _ in images:
        nbi, nbj = 2 * y.shape[0] // B, 2 * y.shape[1] // B
        flat = rng.choice(nbi * nbj, size=min(per, nbi * nbj), replace=False)
        by_image.append([divmod(int(f), nbj) for f in np.sort(flat)])
    n_sample = sum(len(b) for b in by_image)
    cores = min(os.cpu_count() or 1, 16)
    # tasks never mix images (each process caches the per-class matrices of its image)
    chunk = max(1, -(-n_sample // cores))
    tasks = [(k, blocks[i:i + chunk], iters, "RL") for k, blocks in enumerate(by_image)
             for i in range(0, len(blocks), chunk)]
    _ORACLE_IMAGES[:] = images
    try:
        rows, dt = _run_oracle(tasks, cores)
        res = {(k, bi, bj): blk for k, bi, bj, blk, _, _ in rows}
        picks = {(k, bi, bj): pk for k, bi, bj, _, pk, _ in rows}
        gaps = {(k, bi, bj): gp for k, bi, bj, _, _, gp in rows}
        # one core on a part of the same sample, beside the paper's single-core rows
        one = tasks[:max(1, len(tasks) // cores)]
        _, dt1 = _run_oracle(one, 1)
        n_one = sum(len(t[1]) for t in one)
        # the literal L-JSDE form (residual in the measurement domain, no
        # precomputed matrices: the paper's CPU comparison) on a part of the sample
        ltasks, n_l = [], 0
        for k, blocks in enumerate(by_image):
            take = blocks[:max(1, (4 * cores) // len(images))]
            ltasks += [(k, [b], iters, "L") for b in take]
            n_l += len(take)
            if n_l >= 4 * cores:
                break
        _, dt2 = _run_oracle(ltasks, cores)
    finally:
        _ORACLE_IMAGES[:] = []
    rec = {"value": n_sample * B * B / dt / 1e6, "unit": "MP/s", "cores": cores, "kind": "oracle",
           "sample": f"{n_sample} random windows ({n_sample * B * B} px) spread over the {len(images)} image(s) "
                     f"of the {label}, RL-JSDE form (dense per-class B, C, D built per process), {iters} "
                     f"iterations, {dt:.1f} s wall on {cores} processes with 1 BLAS thread each"}
    rec["single_core"] = {"value": n_one * B * B / dt1 / 1e6, "unit": "MP/s",
                          "sample": f"{n_one} of those windows on one process, {dt1:.1f} s"}
    rec["l_jsde_form"] = {"value": n_l * B * B / dt2 / 1e6, "unit": "MP/s",
                          "sample": f"{n_l} of those windows, L-JSDE form, {dt2:.1f} s wall on {cores} processes"}
    rec["cpu_model"] = _cpu_model()
    return rec, res, picks, gaps


def build_inputs(wl: dict):
    if wl["kind"] == "weights":
        wt = random_weights(wl["period"], wl["period"], seed=0)
        clean, observed = synthetic_image(wl["rows"], wl["cols"], seed=0, noise_sigma=wl["noise"])
        return [dict(clean=clean, tile=None, weights=wt, y=sense_weights(observed, wt))]
    if wl["kind"] == "frame":
        return [make_case(wl["rows"], wl["cols"], wl["period"], seed=0, noise=wl["noise"],
                          shape=wl.get("shape", 0xE))]
    return batch_cases(wl["n"], seed=0)


def run_dense(args, wl, cases):
    """The dense form of Sec. IV (FP64, per-class C in device memory): one
    single-image launch per step, the factorised FP64 path timed beside it.
    Its roofline is the FP64 VALU (12 flops per frequency and iteration: the
    metric and the column update of eq. (17)); the HBM side (the distinct C
    columns it reads) is reported beside it."""
    iters = wl["iters"]
    c = cases[0]
    oracle_rec, oracle64_blocks, oracle_picks, oracle_gaps = None, {}, {}, {}
    if not args.no_oracle:
        oracle_rec, oracle64_blocks, oracle_picks, oracle_gaps = cpu_baseline(
            [(c["y"], c["tile"], 0xE, c.get("weights"))], iters, args.oracle_windows,
            label=wl["desc"].split(",")[0])
    import torch
    from paper_2205_02646_amd import ljsde
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    y = torch.from_numpy(c["y"]).to(dev)
    rows, cols = 2 * y.shape[0], 2 * y.shape[1]
    general = c.get("weights") is not None
    pf = None
    if general:  # general layouts run on the dense form only
        pd = ljsde.plan_weights(c["weights"], window=W, block=B, iters=iters, rho=RHO, gamma=GAMMA)
    else:
        pd = ljsde.plan(c["tile"], window=W, block=B, iters=iters, rho=RHO, gamma=GAMMA, fp64=True,
                        dense_c=True)
        if not args.no_fp64:
            pf = ljsde.plan(c["tile"], window=W, block=B, iters=iters, rho=RHO, gamma=GAMMA, fp64=True)
    od = torch.empty((rows, cols), dtype=torch.float64, device=dev)
    of = torch.empty_like(od)

    def timed(fn, steps, warmup):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    if args.profile_copy:
        # a plain device copy of known size (256 MiB read + 256 MiB written):
        # calibrates the HBM byte counters of a profiling run
        a = torch.empty(64 << 20, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    # The first call builds the dense C of the image size (not timed). It also
    # records the selections: the algorithmic HBM bytes are the distinct
    # columns (class, frequency) the launch selects, each read once (windows of
    # a class share their columns), plus the measurements and the output.
    _, sel = ljsde.reconstruct_diag(y, pd, stream=stream)
    torch.cuda.synchronize()
    sel = sel.cpu().numpy().astype(np.int64)
    _, cmap = ljsde.class_map(pd, y.shape[0], y.shape[1])
    keys = cmap.astype(np.int64)[:, None] * (W * W) + sel
    n_cols = int(np.unique(keys[sel >= 0]).size)
    msd = timed(lambda: ljsde.reconstruct(y, pd, out=od, stream=stream), args.steps, max(1, args.warmup))
    msf = None
    if pf is not None:
        msf = timed(lambda: ljsde.reconstruct(y, pf, out=of, stream=stream), max(2, min(args.steps // 4, 5)), 1)
    ljsde.synchronize(stream)
    px = rows * cols
    nwin = (rows // B) * (cols // B)
    o = od.cpu().numpy()
    quality = {}
    if pf is not None:
        quality["maxabs_dense_vs_factorised_fp64"] = float(torch.max(torch.abs(od - of)))
    if oracle64_blocks:
        quality["maxabs_dense_vs_oracle_sample"] = max(
            float(np.max(np.abs(o[B * i:B * i + B, B * j:B * j + B] - blk)))
            for (_, i, j), blk in oracle64_blocks.items())
        quality["oracle_sample_windows"] = len(oracle64_blocks)
        nbj0 = cols // B
        dv = divergence(lambda k: sel[k[1] * nbj0 + k[2]], oracle_picks, oracle_gaps)
        quality["diverged_windows_vs_oracle_sample"] = dv["diverged"]
        quality["diverged_windows_vs_oracle_sample_modulo_conjugation"] = dv["diverged_modulo_conjugation"]
        quality["oracle_top2_gap_at_first_divergence"] = dv["oracle_top2_gap_at_first_divergence"]
        quality["bar_met"] = quality["maxabs_dense_vs_oracle_sample"] <= FP64_TOL
    col_bytes = W * W * 16
    stream_bytes = nwin * iters * col_bytes  # one column of C per window-iteration (eq. (17))
    algo = n_cols * col_bytes + 8 * y.numel() + 8 * px
    hbm_achieved = algo / (msd * 1e-3) / 1e9
    dflops = nwin * iters * W * W * DENSE_FLOPS_PER_FREQ_ITER
    achieved = dflops / (msd * 1e-3)
    rec = {
        "metric": METRIC,
        "value": px / 1e6 / (msd * 1e-3),
        "unit": "MP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": msd,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"RL-JSDE {wl['desc']}, W=32 B=4, {iters} iterations, rho 0.7, gamma 0.5 "
                               "(FP64 single-image launch)",
                   "name": args.workload, "images": 1, "megapixels": px / 1e6, "window": W, "block": B,
                   "iters": iters, "windows": nwin},
        "fp64_plain": None if msf is None else {"value": px / 1e6 / (msf * 1e-3), "unit": "MP/s",
                                                "ms_per_step": msf, "form": "factorised"},
        "quality": quality,
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64_VALU / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_VALU,
                     "algorithmic_flops_per_launch": dflops,
                     "kernel_hash": kernel_hash(DENSE_KERNEL_SOURCES),
                     "hbm": {"achieved_GBps": hbm_achieved, "peak_GBps": HBM_PEAK_GBPS,
                             "frac": hbm_achieved / HBM_PEAK_GBPS,
                             "traffic": load_traffic(args.workload, DENSE_KERNEL_SOURCES),
                             "algorithmic_bytes_per_launch": algo, "distinct_columns": n_cols,
                             "column_stream_GBps": stream_bytes / (msd * 1e-3) / 1e9},
                     "note": "algorithmic flops: 12 per frequency and iteration (the eq. (11) metric 4, the "
                             "eq. (17) column update 8) x W^2 x iterations x windows, against the FP64 vector "
                             "peak. hbm: each distinct FP64 column of C (16 KiB) the launch selects, once, "
                             "plus measurements and output; every window-iteration reads one column "
                             "(column_stream_GBps), repeats are served from L2 / Infinity Cache"},
        "cpu_baseline": oracle_rec,
    }
    print(json.dumps(rec), flush=True)


def run_plain_l(args, wl, cases):
    """Plain L-JSDE (Sec. IV eq. (10) every iteration, residual in the
    measurement domain), FP64, one launch per step, beside the recurrent FP64
    path and the FP32 batched path on the same input: their time ratio is the
    speed-up of the recurrence on this GPU (Sec. V-C compares the same two
    forms). Roofline: the FP64 MFMA peak against the algorithmic flops of the
    eq. (10) product (8 per measurement, frequency and iteration)."""
    iters = wl["iters"]
    c = cases[0]
    oracle_rec, oracle_blocks, oracle_picks, oracle_gaps = None, {}, {}, {}
    if not args.no_oracle:
        oracle_rec, oracle_blocks, oracle_picks, oracle_gaps = cpu_baseline(
            [(c["y"], c["tile"], 0xE, None)], iters, min(args.oracle_windows, 256), label=wl["desc"].split(",")[0])
    import torch
    from paper_2205_02646_amd import ljsde
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    y = torch.from_numpy(c["y"]).to(dev)
    rows, cols = 2 * y.shape[0], 2 * y.shape[1]
    pl = ljsde.plan(c["tile"], window=W, block=B, iters=iters, rho=RHO, gamma=GAMMA, fp64=True, plain_l=True)
    pr = ljsde.plan(c["tile"], window=W, block=B, iters=iters, rho=RHO, gamma=GAMMA, fp64=True)
    p32 = ljsde.plan(c["tile"], window=W, block=B, iters=iters, rho=RHO, gamma=GAMMA, input_f64=True)
    ol = torch.empty((rows, cols), dtype=torch.float64, device=dev)
    orr = torch.empty_like(ol)
    o32 = torch.empty((rows, cols), dtype=torch.float32, device=dev)

    def timed(fn, steps, warmup):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    # the first call builds the basis responses of the image size (not timed)
    # and records the selections
    t0 = time.perf_counter()
    _, sel = ljsde.reconstruct_diag(y, pl, stream=stream)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    sel = sel.cpu().numpy()
    msl = timed(lambda: ljsde.reconstruct(y, pl, out=ol, stream=stream), args.steps, args.warmup)
    msr = timed(lambda: ljsde.reconstruct(y, pr, out=orr, stream=stream), max(3, args.steps), 1)
    ljsde.reconstruct_batch([(y, p32, o32)], stream=stream)
    ms32 = timed(lambda: ljsde.reconstruct_batch([(y, p32, o32)], stream=stream), max(3, args.steps), 1)
    ljsde.synchronize(stream)
    px = rows * cols
    nwin = (rows // B) * (cols // B)
    o = ol.cpu().numpy()
    quality = {"maxabs_plain_l_vs_recurrent_fp64": float(torch.max(torch.abs(ol - orr)))}
    if oracle_blocks:
        quality["maxabs_plain_l_vs_oracle_sample"] = max(
            float(np.max(np.abs(o[B * i:B * i + B, B * j:B * j + B] - blk))) for (_, i, j), blk in oracle_blocks.items())
        quality["oracle_sample_windows"] = len(oracle_blocks)
        nbj0 = cols // B
        dv = divergence(lambda k: sel[k[1] * nbj0 + k[2]], oracle_picks, oracle_gaps)
        quality["diverged_windows_vs_oracle_sample"] = dv["diverged"]
        quality["bar_met"] = quality["maxabs_plain_l_vs_oracle_sample"] <= FP64_TOL and dv["diverged"] == 0
    _, cmap = ljsde.class_map(pl, y.shape[0], y.shape[1])
    n_classes = int(np.unique(cmap).size)
    npos = (W // 2) ** 2
    flops = nwin * iters * 8 * npos * W * W  # eq. (10) numerator: one complex multiply-add per (m, f)
    achieved = flops / (msl * 1e-3)
    rec = {
        "metric": METRIC,
        "value": px / 1e6 / (msl * 1e-3),
        "unit": "MP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": msl,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"plain L-JSDE {wl['desc']}, W=32 B=4, {iters} iterations, rho 0.7, gamma 0.5 "
                               "(FP64 single-image launch)",
                   "name": args.workload, "images": 1, "megapixels": px / 1e6, "window": W, "block": B,
                   "iters": iters, "windows": nwin, "classes": n_classes},
        "recurrent_fp64": {"value": px / 1e6 / (msr * 1e-3), "unit": "MP/s", "ms_per_step": msr},
        "recurrent_fp32_batched": {"value": px / 1e6 / (ms32 * 1e-3), "unit": "MP/s", "ms_per_step": ms32},
        "speedup_recurrent_fp64_vs_plain_l": msl / msr,
        "speedup_recurrent_fp32_batched_vs_plain_l": msl / ms32,
        "setup_ms": {"first_call_with_basis_build": 1e3 * setup_s},
        "quality": quality,
        "roofline": {"bound": "mfma", "achieved": achieved / 1e12, "peak": PEAK_FP64_MFMA / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_MFMA, "traffic": None,
                     "kernel_hash": kernel_hash(["paper_2205_02646_amd/csrc/ljsde_lplain.hip"]),
                     "algorithmic_flops_per_launch": flops,
                     "note": "algorithmic flops: 8 per local measurement, frequency and iteration (the complex "
                             "multiply-add of the eq. (10) numerator) x windows, on FP64 MFMA; windows of one "
                             "local measurement matrix share the product, up to 16 per workgroup, so a "
                             "non-recurrent pattern fills one of the 16 MFMA columns"},
        "cpu_baseline": oracle_rec,
    }
    print(json.dumps(rec), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="batch64", choices=sorted(WORKLOADS))
    ap.add_argument("--oracle-windows", type=int, default=1024)
    ap.add_argument("--no-oracle", action="store_true")
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 path")
    ap.add_argument("--recipe", action="store_true",
                    help="run the reduced-precision recipe instead of the default FP32 plan: FP32 loop state, "
                         "updates and projections, split-BF16 3-term MFMA window DFT with FP32 accumulation "
                         "(FP64 tables, normalisers and stopping test)")
    ap.add_argument("--profile-copy", action="store_true",
                    help="also run a plain device copy of known size (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(windows are independent: a frame would split into strips of block rows, one per GPU)", file=sys.stderr)
        sys.exit(2)

    wl = WORKLOADS[args.workload]
    iters = wl["iters"]
    shape = wl.get("shape", 0xE)
    cases = build_inputs(wl)
    if wl.get("path") == "fp64_dense":
        run_dense(args, wl, cases)
        return
    if wl.get("path") == "plain_l":
        run_plain_l(args, wl, cases)
        return
    # The measurements both paths read: the workload's float64 read-out, or its
    # float32 rounding for a float32 image (frame8192). FP32 plans read float64
    # measurements as they are (LJSDE_INPUT_F64); the oracle runs on the same values.
    y32_input = bool(wl.get("y32"))
    ys = [c["y"].astype(np.float32).astype(np.float64) if y32_input else c["y"] for c in cases]
    label = wl["desc"].split(",")[0] if wl["kind"] == "frame" else "64-image batch"

    oracle_rec, oracle_blocks, oracle_picks, oracle_gaps = (None, {}, {}, {})
    if not args.no_oracle:
        oracle_rec, oracle_blocks, oracle_picks, oracle_gaps = cpu_baseline(
            [(y, c["tile"], shape, None) for y, c in zip(ys, cases)], iters, args.oracle_windows, label=label)

    # the autotuner's choice is read back from its cache file for the report
    import tempfile
    tune_file = os.environ.setdefault("LJSDE_TUNE_CACHE",
                                      os.path.join(tempfile.mkdtemp(prefix="ljsde_tune_"), "tune.json"))

    import torch
    from paper_2205_02646_amd import ljsde

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    jobs, runs64 = [], []
    plan_s = 0.0
    for c, yh in zip(cases, ys):
        rows, cols = 2 * yh.shape[0], 2 * yh.shape[1]
        t0 = time.perf_counter()
        p32 = ljsde.plan(c["tile"], window=W, block=B, iters=iters, rho=RHO, gamma=GAMMA, shape=shape,
                         input_f64=not y32_input, state_fp32=args.recipe, splitbf16=args.recipe)
        plan_s += time.perf_counter() - t0
        y_dev64 = torch.from_numpy(yh).to(dev)
        y_in = y_dev64.to(torch.float32) if y32_input else y_dev64
        jobs.append((y_in, p32, torch.empty((rows, cols), dtype=torch.float32, device=dev)))
        if not args.no_fp64:
            p64 = ljsde.plan(c["tile"], window=W, block=B, iters=iters, rho=RHO, gamma=GAMMA, fp64=True,
                             shape=shape)
            runs64.append((y_dev64, p64, torch.empty((rows, cols), dtype=torch.float64, device=dev)))

    def step32():
        ljsde.reconstruct_batch(jobs, stream=stream)

    def step64():
        for y, pid, out in runs64:
            ljsde.reconstruct(y, pid, out=out, stream=stream)

    def timed(fn, steps, warmup):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps  # ms per step

    # set-up, reported apart from the steps: the first batch call builds the
    # class tables, uploads them, builds the work list and captures the graph
    # (and runs once); the autotuner then times the launch variants
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step32()
    torch.cuda.synchronize()
    first_s = time.perf_counter() - t0
    # pick the launch variant for this batch shape
    t0 = time.perf_counter()
    ljsde.autotune(jobs, stream=stream)
    tune_s = time.perf_counter() - t0
    launch = None
    try:
        with open(tune_file) as fh:
            launch = {k: {"waves_per_workgroup": v[0], "groups_per_claim": v[1], "workgroups_per_cu_below_max": v[2],
                          **({"qd_twiddles": "registers" if v[3] else "lds",
                              "window_dft": "valu" if v[4] else "mfma_f64_16x16x4"} if len(v) > 4 else {})}
                      for k, v in json.load(fh).items()}
    except (OSError, ValueError, IndexError):
        pass

    if args.profile_copy:
        # a plain device copy of known size (256 MiB read + 256 MiB written):
        # calibrates the HBM byte counters of a profiling run
        a = torch.empty(64 << 20, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    # the step is one graph launch on `stream`: its persistent kernel and the
    # one-wavefront counter reset; HIP events on that stream bracket the steps
    ms32 = timed(step32, args.steps, args.warmup)
    ms64 = timed(step64, max(2, min(args.steps // 4, 5)), 1) if runs64 else None
    ljsde.synchronize(stream)

    px = sum(2 * y.shape[0] * 2 * y.shape[1] for y in ys)
    nwin = sum((2 * y.shape[0] // B) * (2 * y.shape[1] // B) for y in ys)
    mp = px / 1e6

    def psnr(err2_sum, n):
        return float(10 * np.log10(255.0 ** 2 / (err2_sum / n)))

    # whole-batch PSNR against the clean images, FP32 and FP64 paths
    o32s = [j[2].cpu().numpy().astype(np.float64) for j in jobs]
    e32 = sum(float(np.sum((o - c["clean"]) ** 2)) for o, c in zip(o32s, cases))
    quality = {"psnr_fp32_db": psnr(e32, px),
               "input": "float32 measurements (float32 image), read by both paths" if y32_input else
                        "float64 measurements, read as they are by both paths"}
    if runs64:
        o64s = [r[2].cpu().numpy() for r in runs64]
        e64 = sum(float(np.sum((o - c["clean"]) ** 2)) for o, c in zip(o64s, cases))
        quality.update({"psnr_fp64_db": psnr(e64, px),
                        "psnr_delta_fp32_vs_fp64_db": abs(psnr(e32, px) - psnr(e64, px)),
                        "maxabs_fp32_vs_fp64": max(float(np.max(np.abs(a - b))) for a, b in zip(o32s, o64s))})
    if oracle_blocks:
        keys = sorted(oracle_blocks)
        g_blk = np.stack([o32s[k][B * i:B * i + B, B * j:B * j + B] for k, i, j in keys])
        r_blk = np.stack([oracle_blocks[key] for key in keys])
        c_blk = np.stack([cases[k]["clean"][B * i:B * i + B, B * j:B * j + B] for k, i, j in keys])

        def psnr_s(a):
            return float(10 * np.log10(255.0 ** 2 / np.mean((a - c_blk) ** 2)))

        # selection sequences of the sampled windows: one diagnostic call per
        # image, which takes the same decisions as the batched kernel
        sels = {}
        for k in sorted({key[0] for key in keys}):
            _, sel = ljsde.reconstruct_diag(jobs[k][0], jobs[k][1], stream=stream)
            torch.cuda.synchronize()
            sels[k] = (sel.cpu().numpy(), 2 * jobs[k][0].shape[1] // B)
        dv = divergence(lambda key: sels[key[0]][0][key[1] * sels[key[0]][1] + key[2]],
                        {key: oracle_picks[key] for key in keys}, oracle_gaps)
        quality.update({"oracle_sample_windows": len(keys),
                        "oracle_sample_images": len({key[0] for key in keys}),
                        "maxabs_fp32_vs_oracle_sample": float(np.max(np.abs(g_blk - r_blk))),
                        "psnr_delta_fp32_vs_oracle_sample_db": abs(psnr_s(g_blk) - psnr_s(r_blk)),
                        "diverged_windows_fp32_vs_oracle_sample": dv["diverged"],
                        "diverged_fraction_fp32_vs_oracle_sample": dv["diverged"] / len(keys),
                        "diverged_windows_fp32_vs_oracle_sample_modulo_conjugation":
                            dv["diverged_modulo_conjugation"],
                        "oracle_top2_gap_at_first_divergence": dv["oracle_top2_gap_at_first_divergence"]})
        if runs64:
            quality["maxabs_fp64_vs_oracle_sample"] = max(
                float(np.max(np.abs(o64s[k][B * i:B * i + B, B * j:B * j + B] - oracle_blocks[(k, i, j)])))
                for k, i, j in keys)
        # the value stands only where the FP32 result holds the parity bar: on
        # the oracle sample, and against the FP64 path on every pixel
        quality["bar_met"] = (quality["maxabs_fp32_vs_oracle_sample"] <= FP32_TOL
                              and quality["psnr_delta_fp32_vs_oracle_sample_db"] <= PSNR_TOL
                              and quality.get("maxabs_fp32_vs_fp64", 0.0) <= FP32_TOL
                              and quality.get("psnr_delta_fp32_vs_fp64_db", 0.0) <= PSNR_TOL)

    flops = nwin * iters * W * W * FLOPS_PER_FREQ_ITER
    achieved = flops / (ms32 * 1e-3)
    ybytes = 4 if y32_input else 8
    # measurements in, float32 image out, and the class tables the kernel reads
    # once per launch: the weighted-mask spectra (FP64), q/D (FP32) and codes
    n_classes = sum(ljsde.class_map(j[1], j[0].shape[0], j[0].shape[1])[0] for j in jobs)
    ws_ = W // 2
    table_bytes = n_classes * (ws_ * ws_ * 4 * 16 + W * W * 4 + ws_ * ws_)
    hbm_bytes = ybytes * sum(y.size for y in ys) + 4 * px + table_bytes
    rec = {
        "metric": METRIC,
        "value": mp / (ms32 * 1e-3),
        "unit": "MP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms32,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"RL-JSDE {wl['desc']}, W=32 B=4, {iters} iterations, rho 0.7, gamma 0.5 "
                               "(FP32 persistent batched launch)",
                   "name": args.workload, "images": len(cases), "megapixels": mp, "window": W, "block": B,
                   "iters": iters, "windows": nwin,
                   "measurements": "float32" if y32_input else "float64"},
        "precision": ("reduced-precision recipe: FP32 loop state, updates, projection, metric and search; "
                      "split-BF16 3-term MFMA window DFT with FP32 accumulation; FP64 tables, normalisers, step "
                      "energy and stopping test" if args.recipe else
                      "FP32 projection, metric and search; FP64 loop state, window DFT (MFMA), step, energy, "
                      "back-transform and near-tie re-decision"),
        "fp64_plain": ({"value": mp / (ms64 * 1e-3), "unit": "MP/s", "ms_per_step": ms64} if ms64 else None),
        # reported only where the FP32 result holds the parity bar (unknown without the oracle)
        "speedup_fp32_batched_vs_fp64_plain": (ms64 / ms32 if ms64 and quality.get("bar_met", True) else None),
        "launch": launch,
        "setup_ms": {"plans": 1e3 * plan_s, "first_batch_call": 1e3 * first_s, "autotune": 1e3 * tune_s},
        "quality": quality,
        "hbm_algorithmic_gbps": hbm_bytes / (ms32 * 1e-3) / 1e9,
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32_VALU / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_VALU,
                     "traffic": None if args.recipe else load_traffic(args.workload), "kernel_hash": kernel_hash(),
                     "algorithmic_flops_per_launch": flops,
                     "algorithmic_hbm_bytes_per_launch": hbm_bytes,
                     "class_tables": {"classes": n_classes, "bytes": table_bytes},
                     "peak_unpacked": PEAK_FP32_VALU / 2e12,
                     "frac_of_peak_unpacked": 2 * achieved / PEAK_FP32_VALU,
                     "lds": {"bytes_per_window_iteration": LDS_BYTES_PER_WIN_ITER,
                             "achieved_TBps": nwin * iters * LDS_BYTES_PER_WIN_ITER / (ms32 * 1e-3) / 1e12,
                             "peak_TBps": PEAK_LDS / 1e12,
                             "frac": nwin * iters * LDS_BYTES_PER_WIN_ITER / (ms32 * 1e-3) / PEAK_LDS},
                     "note": "algorithmic flops: 30 per frequency and iteration (projection 18, metric 4, "
                             "update 8) x W^2 x iterations x windows, over the step time (one graph launch: "
                             "the persistent kernel and its counter reset, HIP events on the launch stream). "
                             "peak: the published FP32 vector peak, which counts packed FP32; this code is "
                             "built with packed FP32 disabled, so its FP32 and FP64 instructions peak at half "
                             "of it (peak_unpacked)"},
        "cpu_baseline": oracle_rec,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
