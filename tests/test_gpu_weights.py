"""GPU parity for general layouts of the 2x2-footprint sensor (Sec. II, eq. (1):
per-pixel quadrant weights; Sec. I: any recurrent layout) and for every
pixel-shape mask, through the C ABI, against the FP64 CPU oracle.

Bar: FP64 <= 1e-9 max-abs, FP32 <= 0.05 grey levels, and equal selection
sequences (ties within a relative 1e-10 go to the lowest frequency index on
both sides; frequencies without any measurement response are never
selected).
"""
import numpy as np
import pytest

from oracle import ljsde_oracle as O
from synth import QUARTER, THREE_QUARTER, make_case, random_pattern, random_weights, sense_weights, \
    shape_weights, synthetic_image

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FP64_TOL = 1e-9
FP32_TOL = 0.05


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2205_02646_amd import ljsde
    ljsde.lib()
    return ljsde


def _dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).to("cuda:0")


def _tile(kind, pr, pc, seed):
    if kind == "random":
        return random_weights(pr, pc, seed=seed)
    if kind == "signed":  # weights of either sign (a difference-of-masks read-out)
        return random_weights(pr, pc, seed=seed) - 0.35
    if kind == "tq01":
        return shape_weights(random_pattern(pr, pc, seed=seed), THREE_QUARTER)
    if kind == "q01":
        return shape_weights(random_pattern(pr, pc, seed=seed), QUARTER)
    if kind == "band":  # no weight on sensor rows 0..8 of a 16-row period
        wt = random_weights(pr, pc, seed=seed)
        wt[:9] = 0.0
        return wt
    raise ValueError(kind)


WCASES = {
    # name: (rows, cols, (pr, pc) or None = whole sensor, kind, W, B, iters, rho, gamma, q_ones, seed)
    "random_w32b4_ragged": (48, 40, (4, 4), "random", 32, 4, 30, 0.7, 0.5, False, 31),
    "random_w16b8": (40, 56, (3, 5), "random", 16, 8, 30, 0.7, 0.5, False, 32),
    "random_w16b4": (24, 40, (2, 3), "random", 16, 4, 40, 0.7, 0.5, False, 33),
    "random_w32b8_qones": (40, 48, (4, 2), "random", 32, 8, 25, 0.6, 1.2, True, 34),
    "signed_w32b4": (40, 40, (3, 3), "signed", 32, 4, 25, 0.7, 0.5, False, 35),
    "random_nonrecurrent": (32, 32, None, "random", 32, 4, 40, 0.7, 0.5, False, 36),
    "tq01_w32b4": (48, 40, (4, 4), "tq01", 32, 4, 30, 0.7, 0.5, False, 37),
    "q01_w16b4": (40, 40, (4, 4), "q01", 16, 4, 30, 0.7, 0.5, False, 38),
    # windows of blocks bi = 2 (mod 8) hold no weighted measurement: no
    # frequency is observed, the first index is picked with a zero step
    "band0_w16b4": (32, 16, (16, 4), "band", 16, 4, 20, 0.7, 0.5, False, 39),
}


def _case(name):
    rows, cols, per, kind, W, B, iters, rho, gamma, q_ones, seed = WCASES[name]
    pr, pc = (rows, cols) if per is None else per
    wt = _tile(kind, pr, pc, seed)
    _, f = synthetic_image(2 * rows, 2 * cols, seed=seed)
    y = sense_weights(f, wt)
    kw = dict(W=W, B=B, iters=iters, rho=rho, gamma=gamma, form="RL", q_mode="ones" if q_ones else "fsr")
    ref, tr = O.reconstruct(y, None, traces=True, weights=wt, **kw)
    return wt, y, ref, tr, dict(window=W, block=B, iters=iters, rho=rho, gamma=gamma, q_ones=q_ones)


@pytest.mark.parametrize("name", list(WCASES))
def test_weights_plan_matches_oracle(L, name):
    wt, y, ref, tr, kw = _case(name)
    pid = L.plan_weights(wt, **kw)
    out, sel = L.reconstruct_diag(_dev(y, np.float64), pid)
    out = out.cpu().numpy()
    sel = sel.cpu().numpy()
    err = np.max(np.abs(out - ref))
    print(f"{name}: weights dense FP64 max-abs {err:.3e}", flush=True)
    assert err <= FP64_TOL
    nbj = out.shape[1] // kw["block"]
    for w in range(sel.shape[0]):
        assert list(sel[w]) == tr[divmod(w, nbj)].picks, w
    # the call without selections runs the same kernel
    out2 = L.reconstruct(_dev(y, np.float64), pid).cpu().numpy()
    assert np.array_equal(out, out2)
    L.release(pid)


@pytest.mark.parametrize("shape", [THREE_QUARTER, QUARTER])
def test_zero_one_weights_match_the_pixel_shape_plan(L, shape):
    """0/1 weights of a code tile give that shape's measurement matrix, so the
    weights plan and the code plan (dense FP64 form) reconstruct the same image
    and select the same frequencies."""
    rows, cols = 40, 48
    tile = random_pattern(4, 4, seed=40 + shape)
    _, f = synthetic_image(2 * rows, 2 * cols, seed=41)
    y = sense_weights(f, shape_weights(tile, shape))
    kw = dict(window=32, block=4, iters=40)
    p_code = L.plan(tile, fp64=True, dense_c=True, shape=0 if shape == THREE_QUARTER else shape, **kw)
    p_wt = L.plan_weights(shape_weights(tile, shape), **kw)
    yd = _dev(y, np.float64)
    a, sa = L.reconstruct_diag(yd, p_code)
    b, sb = L.reconstruct_diag(yd, p_wt)
    err = float((a - b).abs().max())
    print(f"shape 0x{shape:x}: code plan vs weights plan max-abs {err:.3e}", flush=True)
    assert err <= FP64_TOL
    assert torch.equal(sa, sb)
    L.release(p_code)
    L.release(p_wt)


def test_weights_plan_full_size_frame_sampled(L):
    """A 512 x 512 frame (256 x 256 sensor) under a recurrent 4 x 4 general
    layout, in the configuration the benchmark times: sampled target blocks
    (corners, edges, interior) against the oracle, one window at a time."""
    rows = cols = 256
    wt = random_weights(4, 4, seed=50)
    _, f = synthetic_image(2 * rows, 2 * cols, seed=50)
    y = sense_weights(f, wt)
    pid = L.plan_weights(wt, window=32, block=4, iters=100)
    out, sel = L.reconstruct_diag(_dev(y, np.float64), pid)
    out = out.cpu().numpy()
    sel = sel.cpu().numpy()
    nbi = nbj = 2 * rows // 4
    rng = np.random.default_rng(50)
    blocks = [(0, 0), (0, nbj - 1), (nbi - 1, 0), (nbi - 1, nbj - 1), (1, 2), (nbi // 2, 0)]
    blocks += [tuple(int(v) for v in rng.integers(0, nbi, size=2)) for _ in range(10)]
    ref, tr = O.reconstruct(y, None, W=32, B=4, iters=100, form="RL", blocks=blocks, traces=True, weights=wt)
    for bi, bj in blocks:
        blk = (slice(4 * bi, 4 * bi + 4), slice(4 * bj, 4 * bj + 4))
        assert np.max(np.abs(out[blk] - ref[blk])) <= FP64_TOL, (bi, bj)
        assert list(sel[bi * nbj + bj]) == tr[(bi, bj)].picks, (bi, bj)
    assert np.all(np.isfinite(out))
    L.release(pid)


MASK_CASES = {
    # name: (rows, cols, period, W, B, iters, seed, mask)
    "mask7_w32b4": (48, 40, 4, 32, 4, 30, 61, 0x7),    # three quadrants: relabelled three-quarter
    "maskB_w16b8": (40, 56, 4, 16, 8, 30, 62, 0xB),
    "mask4_w32b4": (40, 40, 4, 32, 4, 30, 63, 0x4),    # one quadrant: relabelled quarter
    "half3_w32b4": (48, 40, 4, 32, 4, 30, 64, 0x3),    # horizontal pairs
    "halfA_w16b4": (40, 40, 2, 16, 4, 30, 65, 0xA),    # vertical pairs
    "diag6_w32b8": (40, 48, 4, 32, 8, 25, 66, 0x6),    # diagonal pairs
    "full_w32b4": (40, 40, 4, 32, 4, 25, 67, 0xF),     # full pixels
}


def _mask_case(name):
    rows, cols, per, W, B, iters, seed, mask = MASK_CASES[name]
    c = make_case(rows, cols, per, seed=seed, shape=mask)
    kw = dict(W=W, B=B, iters=iters, form="RL", shape=mask)
    ref, tr = O.reconstruct(c["y"], c["tile"], traces=True, **kw)
    return c, ref, tr, dict(window=W, block=B, iters=iters, shape=mask)


def _check(out, sel, ref, tr, B, tol, label):
    out = out.cpu().numpy().astype(np.float64)
    sel = sel.cpu().numpy()
    err = np.max(np.abs(out - ref))
    print(f"{label}: max-abs {err:.3e}", flush=True)
    assert err <= tol
    nbj = out.shape[1] // B
    for w in range(sel.shape[0]):
        assert list(sel[w]) == tr[divmod(w, nbj)].picks, w


@pytest.mark.parametrize("name", list(MASK_CASES))
def test_every_pixel_shape_matches_oracle(L, name):
    """Masks with three or one collected quadrants run on the three-quarter and
    quarter kernels with relabelled codes (FP64 factorised and dense, FP32);
    two or four collected quadrants run on the general-layout dense form."""
    c, ref, tr, kw = _mask_case(name)
    mask = kw["shape"]
    relabelled = bin(mask).count("1") in (1, 3)
    forms = [dict(fp64=True, dense_c=True)] + ([dict(fp64=True)] if relabelled else [])
    for f in forms:
        pid = L.plan(c["tile"], **f, **kw)
        out, sel = L.reconstruct_diag(_dev(c["y"], np.float64), pid)
        _check(out, sel, ref, tr, kw["block"], FP64_TOL, f"{name} FP64 {'dense' if 'dense_c' in f else 'factorised'}")
        L.release(pid)
    if relabelled:
        y32 = c["y"].astype(np.float32)
        ref32, tr32 = O.reconstruct(y32.astype(np.float64), c["tile"], traces=True, W=kw["window"],
                                    B=kw["block"], iters=kw["iters"], form="RL", shape=mask)
        pid = L.plan(c["tile"], **kw)
        out, sel = L.reconstruct_diag(_dev(y32, np.float32), pid)
        _check(out, sel, ref32, tr32, kw["block"], FP32_TOL, f"{name} FP32")
        L.release(pid)
    else:
        with pytest.raises(L.LjsdeError):
            L.plan(c["tile"], **kw)


@pytest.mark.parametrize("kind,name", [("weights", "random_w32b4_ragged"), ("weights", "random_w16b8"),
                                       ("weights", "band0_w16b4"),
                                       ("mask", "half3_w32b4"), ("mask", "full_w32b4"), ("mask", "mask7_w32b4"),
                                       ("mask", "mask4_w32b4")])
def test_fp32_dense_plans_match_oracle_on_float32_input(L, kind, name):
    """FP32 plans of the dense form: float32 measurements and output, FP64
    arithmetic. Against the oracle run on the same float32 measurements the
    selections are equal and the output differs by its float32 rounding."""
    if kind == "weights":
        rows, cols, per, wkind, W, B, iters, rho, gamma, q_ones, seed = WCASES[name]
        pr, pc = (rows, cols) if per is None else per
        wt = _tile(wkind, pr, pc, seed)
        _, f = synthetic_image(2 * rows, 2 * cols, seed=seed)
        y32 = sense_weights(f, wt).astype(np.float32)
        ref, tr = O.reconstruct(y32.astype(np.float64), None, traces=True, weights=wt, W=W, B=B, iters=iters,
                                rho=rho, gamma=gamma, form="RL", q_mode="ones" if q_ones else "fsr")
        pid = L.plan_weights(wt, window=W, block=B, iters=iters, rho=rho, gamma=gamma, q_ones=q_ones, fp64=False)
    else:
        rows, cols, per, W, B, iters, seed, mask = MASK_CASES[name]
        c = make_case(rows, cols, per, seed=seed, shape=mask)
        y32 = c["y"].astype(np.float32)
        ref, tr = O.reconstruct(y32.astype(np.float64), c["tile"], traces=True, W=W, B=B, iters=iters, form="RL",
                                shape=mask)
        pid = L.plan(c["tile"], window=W, block=B, iters=iters, shape=mask, dense_c=True)
    out, sel = L.reconstruct_diag(_dev(y32, np.float32), pid)
    assert out.dtype == torch.float32
    _check(out, sel, ref, tr, B, 1e-4, f"{name} FP32 dense")
    L.release(pid)


@pytest.mark.parametrize("kind", ["fp64", "fp32_io", "general"])
def test_dense_batch_equals_single_image_calls(L, kind):
    """The dense form over many images in one launch (ljsde_reconstruct_batch
    with dense-form plans): every image equals its single-image dense call
    bitwise, on two consecutive batch calls (the second reuses the batch's
    job table and launch order with new output buffers)."""
    from synth import make_case
    shapes = [(48, 40, 4), (32, 56, 2), (40, 40, (3, 5))]
    items, singles = [], []
    for k, (r, cc, per) in enumerate(shapes):
        if kind == "general":
            wt = random_weights(4, 4, seed=50 + k)
            _, obs = synthetic_image(r, cc, seed=60 + k)
            y = sense_weights(obs, wt)
            pid = L.plan_weights(wt, iters=25)
            ydt, odt = torch.float64, torch.float64
        else:
            c = make_case(r, cc, per, seed=70 + k)
            y = c["y"]
            pid = L.plan(c["tile"], iters=25, fp64=(kind == "fp64"), dense_c=True, input_f64=(kind == "fp32_io"))
            ydt, odt = torch.float64, (torch.float64 if kind == "fp64" else torch.float32)
        yd = torch.from_numpy(np.ascontiguousarray(y)).to("cuda:0").to(ydt)
        items.append((yd, pid, torch.full((r, cc), float("nan"), dtype=odt, device="cuda:0")))
        singles.append(L.reconstruct(yd, pid).clone())
    print(f"dense batch ({kind})", flush=True)
    for rep in range(2):
        if rep:
            items = [(y, pid, torch.full_like(o, float("nan"))) for y, pid, o in items]
        L.reconstruct_batch(items)
        torch.cuda.synchronize()
        for (_, _, o), s in zip(items, singles):
            assert torch.equal(o, s), rep
    for _, pid, _ in items:
        L.release(pid)
