"""GPU parity at the full workload sizes, in the launch configurations the
benchmark times (FP32: persistent batched launch replayed from its graph;
FP64: the plain one-wavefront-per-window launch).

The oracle computes every window of the 512x512 frame, the 256x256 centre
crop of the larger frames (their windows read the full measurements), and
random samples plus border windows elsewhere. Bars: FP64 <= 1e-9 max-abs;
FP32 <= 0.05 max-abs and <= 0.01 dB PSNR delta, no diverged selection
sequence against the oracle on the same input. FP32 plans read the float64
measurements the oracle reads (``input_f64``); the 8192x8192 frame, a float32
image, also runs on float32 measurements against the oracle on those values.
"""
import numpy as np
import pytest

from synth import QUARTER, batch_cases, make_case
from tests.oracle_runs import centre_blocks, run_blocks, run_many, sample_blocks

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FP64_TOL = 1e-9
FP32_TOL = 0.05
B = 4


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2205_02646_amd import ljsde
    ljsde.lib()
    return ljsde


def _canon(k, W=32):
    s, r = divmod(int(k), W)
    return min(s * W + r, ((-s) % W) * W + (-r) % W)


def _psnr(a, b):
    return 10 * np.log10(255.0 ** 2 / np.mean((a - b) ** 2))


def _gather(out, blocks):
    return {(bi, bj): out[B * bi:B * bi + B, B * bj:B * bj + B] for bi, bj in blocks}


def _fp32_batched(L, yh, tile, iters, shape=0):
    """FP32 plan on the persistent batched launch (and its graph replay);
    float64 measurements are read as they are (``input_f64``)."""
    pid = L.plan(tile, iters=iters, shape=shape, input_f64=yh.dtype == np.float64)
    y = torch.from_numpy(yh).to("cuda:0")
    out = torch.empty((2 * yh.shape[0], 2 * yh.shape[1]), dtype=torch.float32, device="cuda:0")
    L.reconstruct_batch([(y, pid, out)])
    L.reconstruct_batch([(y, pid, out)])         # graph replay
    o = out.cpu().numpy().astype(np.float64)
    return pid, y, o


def _fp64_plain(L, y64, tile, iters, shape=0):
    pid = L.plan(tile, iters=iters, fp64=True, shape=shape)
    o = L.reconstruct(torch.from_numpy(y64).to("cuda:0"), pid).cpu().numpy()
    L.release(pid)
    return o


def _fp32_stats(L, pid, y, o32, ref, clean):
    """max-abs, PSNR delta (against the clean image, over the checked blocks)
    and diverged fraction of an FP32 result against the oracle's blocks."""
    blocks = sorted(ref)
    err = max(float(np.max(np.abs(o32[B * i:B * i + B, B * j:B * j + B] - ref[(i, j)][0]))) for i, j in blocks)
    got = np.concatenate([o32[B * i:B * i + B, B * j:B * j + B].ravel() for i, j in blocks])
    exp = np.concatenate([ref[(i, j)][0].ravel() for i, j in blocks])
    cln = np.concatenate([clean[B * i:B * i + B, B * j:B * j + B].ravel() for i, j in blocks])
    dpsnr = abs(_psnr(got, cln) - _psnr(exp, cln))
    _, sel = L.reconstruct_diag(y, pid)
    sel = sel.cpu().numpy()
    nbj = o32.shape[1] // B
    div = np.mean([not np.array_equal(sel[i * nbj + j], ref[(i, j)][1]) for i, j in blocks])
    return err, dpsnr, div


def _check_fp32(L, pid, y, o32, ref, clean, iters, label):
    err, dpsnr, div = _fp32_stats(L, pid, y, o32, ref, clean)
    src = "float64" if y.dtype == torch.float64 else "float32"
    print(f"{label}: FP32 ({src} input) {len(ref)} windows, max-abs {err:.3e}, PSNR delta {dpsnr:.2e} dB, "
          f"diverged {div:.5f}", flush=True)
    assert err <= FP32_TOL
    assert dpsnr <= 0.01
    assert div == 0.0


def _check_fp64(o64, ref, label):
    err = max(float(np.max(np.abs(o64[B * i:B * i + B, B * j:B * j + B] - ref[(i, j)][0]))) for i, j in ref)
    print(f"{label}: FP64 {len(ref)} windows, max-abs {err:.3e}", flush=True)
    assert err <= FP64_TOL


def test_frame512_whole(L):
    """512x512 frame, random 4x4-sensor tile, 100 iterations (the benchmark workload)."""
    c = make_case(512, 512, 4, seed=0)
    blocks = [(i, j) for i in range(128) for j in range(128)]
    ref = run_blocks(c["y"], c["tile"], blocks, iters=100)
    pid, y, o32 = _fp32_batched(L, c["y"], c["tile"], 100)
    _check_fp32(L, pid, y, o32, ref, c["clean"], 100, "frame512")
    L.release(pid)
    _check_fp64(_fp64_plain(L, c["y"], c["tile"], 100), ref, "frame512")


def test_frame512_dense_form_equals_factorised_form(L):
    """The dense form (per-class C of eq. (14), 100 classes) against the
    factorised FP64 path on every window of the 512x512 frame (same selection
    sequences, outputs within the FP64 bar), and against the oracle on a
    sample."""
    c = make_case(512, 512, 4, seed=0)
    y = torch.from_numpy(c["y"]).to("cuda:0")
    pf = L.plan(c["tile"], iters=100, fp64=True)
    pd = L.plan(c["tile"], iters=100, fp64=True, dense_c=True)
    of, sf = L.reconstruct_diag(y, pf)
    od, sd = L.reconstruct_diag(y, pd)
    err = float(torch.max(torch.abs(of - od)))
    same = bool(torch.equal(sf, sd))
    print(f"frame512 dense vs factorised: max-abs {err:.3e}, equal sequences {same}", flush=True)
    assert err <= FP64_TOL and same
    sample = sample_blocks(128, 128, 200, seed=6)
    ref64 = run_blocks(c["y"], c["tile"], sample, iters=100)
    _check_fp64(od.cpu().numpy(), ref64, "frame512 dense")
    L.release(pf)
    L.release(pd)


def test_frame2048_noisy_crop(L):
    """2048x2048 frame with N(0, 2^2) noise, random 8x8-sensor tile, 250 iterations."""
    c = make_case(2048, 2048, 8, seed=0, noise=2.0)
    crop = centre_blocks(512, 512, 256)
    sample = sample_blocks(512, 512, 150, seed=2)
    ref = run_blocks(c["y"], c["tile"], sorted(set(crop) | set(sample)), iters=250)
    pid, y, o32 = _fp32_batched(L, c["y"], c["tile"], 250)
    _check_fp32(L, pid, y, o32, {k: ref[k] for k in crop}, c["clean"], 250, "frame2048 crop")
    L.release(pid)
    _check_fp64(_fp64_plain(L, c["y"], c["tile"], 250), {k: ref[k] for k in sample}, "frame2048")


def test_frame8192_many_classes_crop(L):
    """8192x8192 frame, random 16x16-sensor tile (64 interior classes, 256 with
    the border ones), 250 iterations. A float32 image: the FP32 plan reads
    float32 measurements, and the oracle runs on those same values."""
    c = make_case(8192, 8192, 16, seed=0)
    y32 = c["y"].astype(np.float32)
    crop = centre_blocks(2048, 2048, 256)
    ref32 = run_blocks(y32.astype(np.float64), c["tile"], crop, iters=250)
    pid, y, o32 = _fp32_batched(L, y32, c["tile"], 250)
    _check_fp32(L, pid, y, o32, ref32, c["clean"], 250, "frame8192 crop")
    L.release(pid)
    del y
    sample = sample_blocks(2048, 2048, 100, seed=3)
    ref64 = run_blocks(c["y"], c["tile"], sample, iters=250)
    _check_fp64(_fp64_plain(L, c["y"], c["tile"], 250), ref64, "frame8192")


def test_quarter_sampling_frame1024_crop(L):
    """1024x1024 frame under quarter sampling (one transparent quadrant per
    pixel), random 8x8-sensor tile, 100 iterations: every window of the
    256x256 centre crop and a sample in FP64."""
    c = make_case(1024, 1024, 8, seed=3, shape=QUARTER)
    crop = centre_blocks(256, 256, 256)
    sample = sample_blocks(256, 256, 150, seed=5)
    ref = run_blocks(c["y"], c["tile"], sorted(set(crop) | set(sample)), iters=100, shape=QUARTER)
    pid, y, o32 = _fp32_batched(L, c["y"], c["tile"], 100, shape=QUARTER)
    _check_fp32(L, pid, y, o32, {k: ref[k] for k in crop}, c["clean"], 100, "quarter 1024 crop")
    L.release(pid)
    _check_fp64(_fp64_plain(L, c["y"], c["tile"], 100, shape=QUARTER), {k: ref[k] for k in sample},
                "quarter 1024")


def test_paper_shape_1200(L):
    """The paper's frame shape: 1200x1200, recurrent pattern of period 32 px."""
    c = make_case(1200, 1200, 16, seed=0)
    sample = sample_blocks(300, 300, 600, seed=4)
    ref = run_blocks(c["y"], c["tile"], sample, iters=100)
    pid, y, o32 = _fp32_batched(L, c["y"], c["tile"], 100)
    _check_fp32(L, pid, y, o32, ref, c["clean"], 100, "paper 1200")
    L.release(pid)
    _check_fp64(_fp64_plain(L, c["y"], c["tile"], 100), ref, "paper 1200")


def test_uneven_batch_64_images(L):
    """64 images of uneven size, each with its own pattern of period 2, 4 or 8,
    in one persistent graph-captured launch; 100 iterations, FP32 plans on the
    float64 measurements. Per image, 256 random windows plus border and corner
    windows against the oracle: max-abs, PSNR delta over the checked blocks
    and diverged selection sequences; the plain FP64 path on 8 of the images."""
    cases = batch_cases(64, seed=0)
    items = []
    for k, c in enumerate(cases):
        y = torch.from_numpy(c["y"]).to("cuda:0")
        pid = L.plan(c["tile"], iters=100, input_f64=True)
        out = torch.empty((2 * y.shape[0], 2 * y.shape[1]), dtype=torch.float32, device="cuda:0")
        items.append((y, pid, out))
    L.reconstruct_batch(items)
    L.reconstruct_batch(items)
    torch.cuda.synchronize()
    samples = [sample_blocks(out.shape[0] // B, out.shape[1] // B, 256, seed=10 + k)
               for k, (_, _, out) in enumerate(items)]
    refs = run_many([(c["y"], c["tile"], s) for c, s in zip(cases, samples)], iters=100)
    worst, worst_dpsnr, n_div, n_win = 0.0, 0.0, 0, 0
    for k, (c, (y, pid, out), ref) in enumerate(zip(cases, items, refs)):
        err, dpsnr, div = _fp32_stats(L, pid, y, out.cpu().numpy().astype(np.float64), ref, c["clean"])
        worst, worst_dpsnr = max(worst, err), max(worst_dpsnr, dpsnr)
        n_div += int(round(div * len(ref)))
        n_win += len(ref)
        assert err <= FP32_TOL, (k, err)
        assert dpsnr <= 0.01, (k, dpsnr)
        assert div == 0.0, (k, div)
    print(f"uneven batch: 64 images, {n_win} windows, worst max-abs {worst:.3e}, worst PSNR delta "
          f"{worst_dpsnr:.2e} dB, diverged {n_div}", flush=True)
    for _, pid, _ in items:
        L.release(pid)
    del items
    for k in range(0, 64, 8):
        c = cases[k]
        _check_fp64(_fp64_plain(L, c["y"], c["tile"], 100), refs[k], f"uneven batch image {k}")


DESIGN_NUMBERS = {
    "splitbf16": "the split-BF16 window DFT perturbs the initial state by ~1e-5 relative; on the 512x512 "
                 "frame 11% of the windows then pick a different sequence (near ties with top-2 gaps "
                 "0..6.6e-4), up to 8.3 grey levels",
    "state_fp32": "the FP32 loop state drifts by ~1e-5 relative over 100 iterations; on the 512x512 frame "
                  "0.085% of the windows flip a near tie (top-2 gaps 6.9e-9..6.7e-6), up to 2.5 grey levels",
    "recipe": "both together (FP32 state, updates and projections; split-BF16 window DFT): the two "
              "perturbations add up",
}
VARIANT_FLAGS = {"splitbf16": dict(splitbf16=True), "state_fp32": dict(state_fp32=True),
                 "recipe": dict(state_fp32=True, splitbf16=True)}


@pytest.mark.parametrize("variant", ["splitbf16", "state_fp32", "recipe"])
@pytest.mark.xfail(strict=True, reason="reduced-precision options miss the 0.05 max-abs bar")
def test_frame512_reduced_precision_options_hold_the_fp32_bar(L, variant):
    """The reduced-precision options (split-BF16 window DFT; FP32 loop state;
    both together, the brief's full recipe) against the FP32 bar on the whole
    512x512 frame: max-abs <= 0.05, PSNR
    delta <= 0.01 dB, no diverged selection sequence. Expected to fail (strict
    xfail, so that a fix shows): greedy selection is discontinuous, and their
    rounding flips near ties. The numbers are printed."""
    c = make_case(512, 512, 4, seed=0)
    blocks = [(i, j) for i in range(128) for j in range(128)]
    ref = run_blocks(c["y"], c["tile"], blocks, iters=100)
    pid = L.plan(c["tile"], iters=100, input_f64=True, **VARIANT_FLAGS[variant])
    y = torch.from_numpy(c["y"]).to("cuda:0")
    out = torch.empty((512, 512), dtype=torch.float32, device="cuda:0")
    L.reconstruct_batch([(y, pid, out)])
    o = out.cpu().numpy().astype(np.float64)
    exp = np.zeros_like(o)
    for (i, j), (blk, _, _) in ref.items():
        exp[B * i:B * i + B, B * j:B * j + B] = blk
    err = np.abs(o - exp).reshape(128, 4, 128, 4).max(axis=(1, 3))
    dpsnr = abs(_psnr(o, c["clean"]) - _psnr(exp, c["clean"]))
    # diverged selection sequences: raw, modulo conjugate partners (which give
    # the same real output), and the oracle's top-2 gap at the first divergence
    _, sel = L.reconstruct_diag(y, pid)
    sel = sel.cpu().numpy()
    raw, canon, gaps = 0, 0, []
    for (i, j), (_, picks, gap) in ref.items():
        s = sel[i * 128 + j]
        if np.array_equal(s, picks):
            continue
        raw += 1
        gaps.append(float(gap[int(np.flatnonzero(s != picks)[0])]))
        canon += [_canon(k) for k in s] != [_canon(k) for k in picks]
    n = len(ref)
    gap_txt = f", top-2 gap at first divergence {min(gaps):.1e}..{max(gaps):.1e}" if gaps else ""
    print(f"{variant}: max-abs {err.max():.3e}, windows above 0.05: {np.mean(err > 0.05):.5f}, "
          f"PSNR delta {dpsnr:.2e} dB, diverged windows {raw / n:.5f} (modulo conjugation {canon / n:.5f})"
          f"{gap_txt} [{DESIGN_NUMBERS[variant]}]", flush=True)
    L.release(pid)
    assert dpsnr <= 0.01
    assert err.max() <= FP32_TOL
    assert raw == 0
