"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Bars (fixed by the project goal): FP64 mode <= 1e-9 max-abs; FP32 mode
<= 0.05 grey levels max-abs and <= 0.01 dB PSNR delta. FP32 plans run on the
same float64 measurements as the oracle (plans with ``input_f64``), and also
on float32 measurements, against the oracle run on those same values (rounded
to float32, then computed in FP64). Selection sequences must be equal: ties
(metrics within a relative 1e-10) go to the lowest frequency index on both
sides. The all-FP32 variant decides in FP32 and is held to the output bars
only.
"""
import numpy as np
import pytest

from oracle import ljsde_oracle as O
from synth import QUARTER, THREE_QUARTER, make_case, random_pattern, sense

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


def _canon(k, W):
    s, r = divmod(int(k), W)
    return min(s * W + r, ((-s) % W) * W + (-r) % W)


def _psnr(a, b):
    return 10 * np.log10(255.0 ** 2 / np.mean((a - b) ** 2))


TQ, QS = THREE_QUARTER, QUARTER
CASES = {
    # name: (rows, cols, pattern, W, B, iters, rho, gamma, q_ones, seed, pixel shape)
    "w32b4_ragged": (48, 40, 4, 32, 4, 30, 0.7, 0.5, False, 5, TQ),
    "nonrecurrent_64": (64, 64, None, 32, 4, 100, 0.7, 0.5, False, 0, TQ),
    "w16b4": (40, 56, (3, 5), 16, 4, 40, 0.7, 0.5, False, 6, TQ),
    "w32b8": (48, 64, 4, 32, 8, 25, 0.7, 0.5, False, 7, TQ),
    "q_ones": (40, 40, 4, 32, 4, 25, 0.7, 0.5, True, 8, TQ),
    "gamma_rho": (40, 48, 2, 32, 4, 25, 0.5, 1.5, False, 9, TQ),
    "w16b8_tiny": (8, 24, 2, 16, 8, 12, 0.7, 0.5, False, 10, TQ),
    # a whole image of one target block (one window, mostly outside the image)
    "one_block_w32b4": (4, 4, None, 32, 4, 20, 0.7, 0.5, False, 14, TQ),
    "one_block_w16b8": (8, 8, None, 16, 8, 15, 0.7, 0.5, False, 15, TQ),
    "single_iteration": (24, 24, 4, 32, 4, 1, 0.7, 0.5, False, 16, TQ),
    # quarter sampling (one transparent quadrant per pixel)
    "quarter_w32b4": (48, 40, 4, 32, 4, 30, 0.7, 0.5, False, 11, QS),
    "quarter_nonrecurrent": (64, 64, None, 32, 4, 60, 0.7, 0.5, False, 12, QS),
    "quarter_w16b8": (40, 56, (3, 5), 16, 8, 30, 0.7, 0.5, False, 13, QS),
    # more picks than the FP32 kernel keeps at once for eq. (18) (W^2 / 4:
    # 64 at W = 16, 256 at W = 32), so its running sums are taken mid-window
    "w16b4_long": (40, 56, (3, 5), 16, 4, 150, 0.7, 0.5, False, 17, TQ),
    "w32b4_long": (32, 40, 4, 32, 4, 260, 0.7, 0.5, False, 18, TQ),
}


def _case(name):
    rows, cols, pattern, W, B, iters, rho, gamma, q_ones, seed, shape = CASES[name]
    c = make_case(rows, cols, pattern, seed=seed, shape=shape)
    kw = dict(W=W, B=B, iters=iters, rho=rho, gamma=gamma, form="RL", q_mode="ones" if q_ones else "fsr",
              shape=shape)
    ref, tr = O.reconstruct(c["y"], c["tile"], traces=True, **kw)
    c["y32"] = c["y"].astype(np.float32)
    c["ref32"], c["tr32"] = O.reconstruct(c["y32"].astype(np.float64), c["tile"], traces=True, **kw)
    return c, ref, tr, dict(window=W, block=B, iters=iters, rho=rho, gamma=gamma, q_ones=q_ones,
                            shape=0 if shape == TQ else shape)


_cache = {}


def _cached(name):
    if name not in _cache:
        _cache[name] = _case(name)
    return _cache[name]


@pytest.mark.parametrize("dense", [False, True], ids=["factorised", "denseC"])
@pytest.mark.parametrize("name", list(CASES))
def test_fp64_matches_oracle(L, name, dense):
    """FP64 plans, in the factorised form and in the dense form (per-class C
    of eq. (14) in device memory, R as the state)."""
    c, ref, tr, kw = _cached(name)
    pid = L.plan(c["tile"], fp64=True, dense_c=dense, **kw)
    out, sel = L.reconstruct_diag(_dev(c["y"], np.float64), pid)
    out = out.cpu().numpy()
    sel = sel.cpu().numpy()
    err = np.max(np.abs(out - ref))
    print(f"{name}: FP64 {'dense C' if dense else 'factorised'} max-abs {err:.3e}")
    assert err <= FP64_TOL
    W = kw["window"]
    nbj = out.shape[1] // kw["block"]
    for w in range(sel.shape[0]):
        assert list(sel[w]) == tr[divmod(w, nbj)].picks, w
    L.release(pid)


@pytest.mark.parametrize("input_f64", [True, False], ids=["f64in", "f32in"])
@pytest.mark.parametrize("state_fp32", [False, True], ids=["fp64state", "fp32state"])
@pytest.mark.parametrize("name", list(CASES))
def test_fp32_matches_oracle(L, name, state_fp32, input_f64):
    """FP32 plans against the FP64 oracle on the same measurements: float64
    (the oracle's own input) or float32."""
    if state_fp32 and CASES[name][-1] != THREE_QUARTER:
        pytest.skip("the all-FP32 variant exists for three-quarter sampling only")
    if state_fp32 and name.endswith("_long"):
        pytest.skip("the FP32 state drifts over hundreds of iterations; the precision options are bounded "
                    "at full size under a strict xfail")
    c, ref, tr, kw = _cached(name)
    if input_f64:
        y, ydt, ref_out, ref_tr = c["y"], np.float64, ref, tr
    else:
        y, ydt, ref_out, ref_tr = c["y32"], np.float32, c["ref32"], c["tr32"]
    pid = L.plan(c["tile"], state_fp32=state_fp32, input_f64=input_f64, **kw)
    out, sel = L.reconstruct_diag(_dev(y, ydt), pid)
    out_b = L.reconstruct(_dev(y, ydt), pid)          # batched persistent path
    assert out.dtype == torch.float32
    assert torch.equal(out, out_b)
    out = out.cpu().numpy().astype(np.float64)
    sel = sel.cpu().numpy()
    err = np.max(np.abs(out - ref_out))
    dpsnr = abs(_psnr(out, c["clean"]) - _psnr(ref_out, c["clean"]))
    W = kw["window"]
    nbj = out.shape[1] // kw["block"]
    div = np.mean([list(sel[w]) != ref_tr[divmod(w, nbj)].picks for w in range(sel.shape[0])])
    print(f"{name}: FP32 ({'float64' if input_f64 else 'float32'} input) max-abs {err:.3e}, "
          f"PSNR delta {dpsnr:.2e} dB, diverged windows {div:.4f}")
    assert err <= FP32_TOL
    assert dpsnr <= 0.01
    if not state_fp32:
        assert div == 0.0
    L.release(pid)


def test_quarter_sampling_batch_equals_single_and_graph_replays(L):
    """The same for quarter sampling: uneven images of one pixel shape and
    different pattern periods in one persistent launch, replayed from its graph
    with eager work between the replays; every replay equals the single-image
    (diagnostic-kernel) run."""
    shapes = [(48, 40, 2), (32, 56, 4), (24, 24, 8)]
    items, singles = [], []
    for k, (r, cc, per) in enumerate(shapes):
        case = make_case(r, cc, per, seed=40 + k, shape=QS)
        pid = L.plan(case["tile"], iters=25, shape=QS, input_f64=True)
        y = _dev(case["y"], np.float64)
        out = torch.empty((r, cc), dtype=torch.float32, device="cuda:0")
        items.append((y, pid, out))
        singles.append(L.reconstruct_diag(y, pid)[0].clone())
    for rep in range(3):
        for _, _, out in items:
            out.fill_(float("nan"))
        L.reconstruct_batch(items)
        torch.cuda.synchronize()
        _ = torch.ones(1000, device="cuda:0").sum().item()
        for (y, pid, out), s in zip(items, singles):
            assert torch.equal(out, s), rep
    for _, pid, _ in items:
        L.release(pid)


@pytest.mark.parametrize("state_fp32", [False, True], ids=["fp64state", "fp32state"])
def test_batch_equals_single_and_graph_replays(L, state_fp32):
    """Uneven images, different patterns and periods, one persistent launch
    replayed from its graph; every replay equals the single-image run."""
    shapes = [(40, 48, 2), (64, 40, 4), (24, 24, 8), (48, 72, 4)]
    items, singles = [], []
    for k, (r, cc, per) in enumerate(shapes):
        case = make_case(r, cc, per, seed=20 + k)
        pid = L.plan(case["tile"], iters=20, state_fp32=state_fp32)
        y = _dev(case["y"], np.float32)
        out = torch.empty((r, cc), dtype=torch.float32, device="cuda:0")
        items.append((y, pid, out))
        singles.append(L.reconstruct_diag(y, pid)[0].clone())
    for rep in range(4):
        for _, _, out in items:
            out.fill_(float("nan"))
        L.reconstruct_batch(items)
        torch.cuda.synchronize()
        # eager work between replays
        _ = torch.ones(1000, device="cuda:0").sum().item()
        for (y, pid, out), s in zip(items, singles):
            assert torch.equal(out, s), rep
    for _, pid, _ in items:
        L.release(pid)


def test_fp32_is_deterministic(L):
    c, ref, tr, kw = _cached("nonrecurrent_64")
    pid = L.plan(c["tile"], **kw)
    y = _dev(c["y"], np.float32)
    a = L.reconstruct(y, pid).clone()
    b = L.reconstruct(y, pid).clone()
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    L.release(pid)


def test_constant_image_closed_form_on_gpu(L):
    """f = c: every window picks DC, f-hat = (1 - (1 - gamma)^K) c. The picks
    are checked over the first 12 iterations only: later the residual is a
    few ulps of the initial one and rounding decides the argmax (the output
    is unaffected at that level)."""
    tile = random_pattern(4, 4, seed=4)
    y = sense(np.full((40, 48), 100.0), tile)
    for fp64, tol in ((True, 1e-10), (False, 1e-3)):
        dt = np.float64 if fp64 else np.float32
        pid = L.plan(tile, iters=30, fp64=fp64)
        out = L.reconstruct(_dev(y, dt), pid)
        np.testing.assert_allclose(out.cpu().numpy(), (1 - 0.5 ** 30) * 100.0, atol=tol)
        L.release(pid)
        pid = L.plan(tile, iters=12, fp64=fp64)
        out, sel = L.reconstruct_diag(_dev(y, dt), pid)
        np.testing.assert_allclose(out.cpu().numpy(), (1 - 0.5 ** 12) * 100.0, atol=tol)
        assert (sel.cpu().numpy() == 0).all()
        L.release(pid)


@pytest.mark.parametrize("form", ["fp64", "fp64_dense", "fp32", "fp32_dense", "fp32_batched"])
def test_zero_measurements_give_a_zero_image_and_dc_picks(L, form):
    """y = 0: every metric of eq. (11) is 0, so every pick is the lowest index
    (DC, by the tie rule), every step is 0 and the image is 0; the oracle
    agrees. With an energy floor the window stops after its first pick."""
    tile = random_pattern(4, 4, seed=9)
    y = np.zeros((20, 24))
    ref, tr = O.reconstruct(y, tile, W=32, B=4, iters=10, form="RL", traces=True)
    assert all(t.picks == [0] * 10 for t in tr.values()) and not ref.any()
    fp64 = form.startswith("fp64")
    dt = np.float64 if fp64 else np.float32
    pid = L.plan(tile, iters=10, fp64=fp64, dense_c=form.endswith("dense"))
    if form == "fp32_batched":
        out = L.reconstruct(_dev(y, dt), pid)
        assert not out.cpu().numpy().any()
    else:
        out, sel = L.reconstruct_diag(_dev(y, dt), pid)
        assert not out.cpu().numpy().any()
        assert (sel.cpu().numpy() == 0).all()
        L.set_energy_floor(pid, 0.5)
        out, sel = L.reconstruct_diag(_dev(y, dt), pid)
        sel = sel.cpu().numpy()
        assert (sel[:, 0] == 0).all() and (sel[:, 1:] == -1).all()
    L.release(pid)


@pytest.mark.parametrize("form", ["fp64", "fp64_dense", "fp32", "fp32_dense"])
def test_energy_floor_stops_early_like_a_shorter_oracle_run(L, form):
    """The optional energy floor: a window stops after the first iteration
    whose weighted residual energy (eq. (8), from the oracle's L-JSDE
    residual) is at most tau times its initial value, and its output is that
    of the shorter oracle run."""
    tau = 0.02
    c = make_case(40, 40, 4, seed=31)
    fp64 = form.startswith("fp64")
    y = c["y"] if fp64 else c["y"].astype(np.float32).astype(np.float64)
    pid = L.plan(c["tile"], iters=60, fp64=fp64, dense_c=form.endswith("dense"))
    L.set_energy_floor(pid, tau)
    out, sel = L.reconstruct_diag(_dev(y, np.float64 if fp64 else np.float32), pid)
    out = out.cpu().numpy().astype(np.float64)
    sel = sel.cpu().numpy()
    n_done = (sel >= 0).sum(axis=1)
    assert n_done.min() < 60                        # some windows stopped
    assert all((sel[w, n:] == -1).all() for w, n in enumerate(n_done))
    nbj = 40 // 4
    tol = FP64_TOL if form == "fp64" or form == "fp64_dense" else 1e-4
    for w in range(sel.shape[0]):
        bi, bj = divmod(w, nbj)
        _, trL = O.reconstruct(y, c["tile"], iters=60, form="L", blocks=[(bi, bj)], traces=True)
        t = trL[(bi, bj)]
        stop = next((k + 1 for k, e in enumerate(t.energy) if e <= tau * t.energy0), 60)
        assert n_done[w] == stop, (w, n_done[w], stop)
        ref = O.reconstruct(y, c["tile"], iters=int(n_done[w]), form="RL", blocks=[(bi, bj)])
        blk = np.s_[4 * bi:4 * bi + 4, 4 * bj:4 * bj + 4]
        assert np.max(np.abs(out[blk] - ref[blk])) <= tol
    L.release(pid)


def test_splitbf16_dft_accuracy_after_one_iteration(L):
    """The split-BF16 window DFT has a relative error of ~2^-16: after one
    iteration (one pick and step per window) the outputs match the oracle to
    ~1e-4 of their scale wherever the pick agrees, and the pick agrees in all
    but rare near ties."""
    c = make_case(128, 128, 4, seed=41)
    y32 = c["y"].astype(np.float32)
    ref, tr = O.reconstruct(y32.astype(np.float64), c["tile"], iters=1, form="RL", traces=True)
    pid = L.plan(c["tile"], iters=1, splitbf16=True)
    out, sel = L.reconstruct_diag(_dev(y32, np.float32), pid)
    out = out.cpu().numpy().astype(np.float64)
    sel = sel.cpu().numpy()
    nbj = 128 // 4
    same = [w for w in range(sel.shape[0]) if sel[w, 0] == tr[divmod(w, nbj)].picks[0]]
    assert len(same) >= 0.99 * sel.shape[0]
    scale = np.max(np.abs(ref))
    err = max(np.max(np.abs(out[4 * (w // nbj):4 * (w // nbj) + 4, 4 * (w % nbj):4 * (w % nbj) + 4]
                             - ref[4 * (w // nbj):4 * (w // nbj) + 4, 4 * (w % nbj):4 * (w % nbj) + 4]))
              for w in same)
    print(f"split-BF16, 1 iteration: {len(same)}/{sel.shape[0]} equal picks, max-abs {err:.3e} (scale {scale:.1f})")
    assert err <= 2e-4 * scale
    L.release(pid)


def test_autotune_keeps_results_and_writes_its_cache(L, tmp_path, monkeypatch):
    """Every launch variant the autotuner times computes each window the same
    way: the batch gives bitwise the same images before and after tuning, and
    the choice is written to the file named by LJSDE_TUNE_CACHE."""
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("LJSDE_TUNE_CACHE", str(cache))
    items = []
    for k, (r, cc, per) in enumerate([(40, 56, 2), (64, 48, 4), (24, 32, 8)]):
        case = make_case(r, cc, per, seed=60 + k)
        pid = L.plan(case["tile"], iters=25)
        items.append((_dev(case["y"].astype(np.float32), np.float32), pid,
                      torch.empty((r, cc), dtype=torch.float32, device="cuda:0")))
    L.reconstruct_batch(items)
    before = [o.clone() for _, _, o in items]
    L.autotune(items)
    for _, _, o in items:
        o.zero_()
    L.reconstruct_batch(items)
    torch.cuda.synchronize()
    import json
    tuned = json.loads(cache.read_text())
    assert len(tuned) >= 1
    for v in tuned.values():
        # windows per workgroup, groups per claim, fewer workgroups per CU,
        # q/D and twiddles in registers, VALU window DFT
        assert len(v) == 5 and v[0] in (1, 2, 4) and v[1] in (1, 2, 4) and v[2] in (0, 1)
        assert v[3] in (0, 1) and v[4] in (0, 1)
    vdft = any(v[4] for v in tuned.values())
    for b, (_, _, o) in zip(before, items):
        # the VALU DFT sums in another order (FP64): equal up to rounding
        assert torch.equal(b, o) if not vdft else float(torch.max(torch.abs(b - o))) <= 1e-3
    for _, pid, _ in items:
        L.release(pid)


@pytest.mark.parametrize("variant", ["1,1,0,0,0", "2,2,0,0,0", "4,4,1,0,0", "4,1,0,1,0", "2,4,0,1,0",
                                     "4,1,0,0,1", "1,2,1,1,1"])
def test_every_launch_variant_gives_the_same_images(L, monkeypatch, variant):
    """The autotuner's knobs (windows per workgroup, groups per claim,
    resident workgroups per CU, q/D and twiddles in registers or LDS, window
    DFT on FP64 MFMA or as VALU passes), forced one at a time: the batched
    images equal the diagnostic single-image calls bitwise, and within FP64
    rounding of the DFT's summation order for the VALU DFT."""
    monkeypatch.setenv("LJSDE_VARIANT", variant)
    vdft = variant.endswith(",1")
    items, singles = [], []
    for k, (r, cc, per) in enumerate([(96, 80, 2), (64, 120, 4), (72, 72, 8), (40, 48, 4)]):
        case = make_case(r, cc, per, seed=90 + k)
        pid = L.plan(case["tile"], iters=30, input_f64=True)
        y = _dev(case["y"], np.float64)
        items.append((y, pid, torch.full((r, cc), float("nan"), dtype=torch.float32, device="cuda:0")))
        singles.append(L.reconstruct_diag(y, pid)[0].clone())
    print(f"launch variant {variant}", flush=True)
    for rep in range(2):
        L.reconstruct_batch(items)
        torch.cuda.synchronize()
        for (_, _, o), s in zip(items, singles):
            if vdft:
                assert float(torch.max(torch.abs(o - s))) <= 1e-3
            else:
                assert torch.equal(o, s), rep
    # the allocation-free call takes the forced variant too
    y, pid, o = items[0]
    out = torch.full_like(o, float("nan"))
    L.reconstruct_noalloc(y, pid, out)
    torch.cuda.synchronize()
    assert torch.equal(out, o)
    for _, pid, _ in items:
        L.release(pid)


def test_calls_on_two_streams_may_overlap(L):
    """The same batch launched on two streams without a wait in between (each
    stream has its own work counters and job table), and a dense-form plan
    whose first call builds C on one stream while the next call runs on
    another: every image equals its single-stream result."""
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    items, refs = [], []
    for k, (r, cc, per) in enumerate([(48, 64, 4), (32, 40, 2)]):
        case = make_case(r, cc, per, seed=80 + k)
        pid = L.plan(case["tile"], iters=40)
        y = _dev(case["y"].astype(np.float32), np.float32)
        items.append((y, pid))
        refs.append(L.reconstruct(y, pid))
    torch.cuda.synchronize()
    outs = []
    for st in (s1, s2):
        jobs = [(y, pid, torch.empty((2 * y.shape[0], 2 * y.shape[1]), dtype=torch.float32, device="cuda:0"))
                for y, pid in items]
        L.reconstruct_batch(jobs, stream=st)
        outs.append([o for _, _, o in jobs])
    torch.cuda.synchronize()
    for per_stream in outs:
        for ref, o in zip(refs, per_stream):
            assert torch.equal(ref, o)
    for _, pid in items:
        L.release(pid)
    # dense form: C is complete before a call on another stream can read it
    case = make_case(256, 256, 4, seed=83)
    pid = L.plan(case["tile"], iters=30, fp64=True, dense_c=True)
    y = _dev(case["y"], np.float64)
    o1 = L.reconstruct(y, pid, stream=s1)
    o2 = L.reconstruct(y, pid, stream=s2)
    torch.cuda.synchronize()
    assert torch.equal(o1, o2)
    blocks = [(0, 0), (31, 17), (63, 63)]
    ref = O.reconstruct(case["y"], case["tile"], iters=30, form="RL", blocks=blocks)
    o = o2.cpu().numpy()
    for bi, bj in blocks:
        blk = np.s_[4 * bi:4 * bi + 4, 4 * bj:4 * bj + 4]
        assert np.max(np.abs(o[blk] - ref[blk])) <= FP64_TOL
    L.release(pid)


@pytest.mark.parametrize("form", ["fp64", "fp64_dense", "fp32_batched"])
def test_failed_allocation_reports_enomem_and_leaves_no_partial_state(L, form, monkeypatch):
    """A device allocation that fails (simulated: LJSDE_FAULT=alloc) is
    reported as LJSDE_ENOMEM, and the next call, with memory available, builds
    everything it needs and returns the right image."""
    case = make_case(32, 40, 4, seed=90)
    fp64 = form.startswith("fp64")
    y = case["y"] if fp64 else case["y"].astype(np.float32).astype(np.float64)
    pid = L.plan(case["tile"], iters=20, fp64=fp64, dense_c=form == "fp64_dense")
    yd = _dev(y, np.float64 if fp64 else np.float32)
    monkeypatch.setenv("LJSDE_FAULT", "alloc")
    with pytest.raises(L.LjsdeError) as e:
        L.reconstruct(yd, pid)
    assert e.value.code == L.ENOMEM
    monkeypatch.delenv("LJSDE_FAULT")
    out = L.reconstruct(yd, pid).cpu().numpy().astype(np.float64)
    ref = O.reconstruct(y, case["tile"], iters=20, form="RL")
    assert np.max(np.abs(out - ref)) <= (FP64_TOL if fp64 else 0.05)
    L.release(pid)


def test_host_buffers_are_refused_before_any_launch(L):
    """Measurements and output must be device memory: the binding refuses CPU
    tensors, and the C ABI itself refuses host pointers (LJSDE_EINVAL, no
    kernel launched), for single calls and batches; a valid call afterwards
    runs normally."""
    import ctypes
    c = make_case(24, 24, 4, seed=90)
    y = _dev(c["y"].astype(np.float32), np.float32)
    pid = L.plan(c["tile"], iters=10)
    good = L.reconstruct(y, pid).cpu().numpy()
    with pytest.raises(TypeError):
        L.reconstruct(y, pid, out=torch.empty((24, 24), dtype=torch.float32))
    with pytest.raises(TypeError):
        L.reconstruct(y.cpu(), pid)
    with pytest.raises(TypeError):
        L.reconstruct_batch([(y, pid, torch.empty((24, 24), dtype=torch.float32))])
    host = np.zeros((24, 24), np.float32)
    hp = ctypes.c_void_p(host.ctypes.data)
    lib = L.lib()
    assert lib.ljsde_reconstruct(y.data_ptr(), 12, 12, pid, hp, None) == L.EINVAL
    assert "not" in L.last_error() and "device" in L.last_error()
    assert lib.ljsde_reconstruct(hp, 12, 12, pid, y.data_ptr(), None) == L.EINVAL
    jobs = (L.Job * 1)(L.Job(y.data_ptr(), 12, 12, pid, host.ctypes.data))
    assert lib.ljsde_reconstruct_batch(jobs, 1, None) == L.EINVAL
    assert lib.ljsde_reconstruct_batch(jobs, 1, None) == L.EINVAL   # checked again, not cached
    torch.cuda.synchronize()
    assert np.array_equal(L.reconstruct(y, pid).cpu().numpy(), good)
    assert not np.any(host)
    L.release(pid)


def test_element_type_follows_the_plan(L):
    """The binding takes the element type from the plan (float32 for FP32
    plans, float64 for FP64 plans), so a tensor of the other type is refused
    instead of being read with the wrong width."""
    c = make_case(24, 24, 4, seed=91)
    p32 = L.plan(c["tile"], iters=5)
    p64 = L.plan(c["tile"], iters=5, fp64=True)
    y32 = _dev(c["y"].astype(np.float32), np.float32)
    y64 = _dev(c["y"], np.float64)
    with pytest.raises(TypeError):
        L.reconstruct(y64, p32)
    with pytest.raises(TypeError):
        L.reconstruct(y32, p64)
    with pytest.raises(TypeError):
        L.reconstruct(y32, p32, fp64=True)
    with pytest.raises(TypeError):
        L.reconstruct_batch([(y32, p64, torch.empty((24, 24), dtype=torch.float32, device="cuda:0"))])
    assert L.reconstruct(y32, p32).dtype == torch.float32
    assert L.reconstruct(y64, p64).dtype == torch.float64
    # FP32 plans made with input_f64 read float64 measurements, write float32
    pin = L.plan(c["tile"], iters=5, input_f64=True)
    with pytest.raises(TypeError):
        L.reconstruct(y32, pin)
    with pytest.raises(TypeError):
        L.reconstruct_batch([(y32, pin, torch.empty((24, 24), dtype=torch.float32, device="cuda:0"))])
    assert L.reconstruct(y64, pin).dtype == torch.float32
    L.release(p32)
    L.release(p64)
    L.release(pin)


def test_batch_mixes_float32_and_float64_measurements(L):
    """One batch whose jobs read float32 and float64 measurements (by their
    plans) gives each job the result of its single-image call."""
    cases = [make_case(r, c, p, seed=60 + k) for k, (r, c, p) in enumerate([(40, 48, 4), (24, 36, 2), (32, 32, 8)])]
    items, singles = [], []
    for k, c in enumerate(cases):
        f64 = k % 2 == 0
        pid = L.plan(c["tile"], iters=20, input_f64=f64)
        y = _dev(c["y"], np.float64) if f64 else _dev(c["y"].astype(np.float32), np.float32)
        out = torch.empty((2 * y.shape[0], 2 * y.shape[1]), dtype=torch.float32, device="cuda:0")
        items.append((y, pid, out))
        singles.append(L.reconstruct_diag(y, pid)[0])
    L.reconstruct_batch(items)
    torch.cuda.synchronize()
    for (y, pid, out), ref in zip(items, singles):
        assert torch.equal(out, ref)
        L.release(pid)


def test_energy_floor_change_reaches_the_batched_path(L):
    """A batched call, then a new energy floor, then another batched call: the
    second call honours the new floor (equal to the diagnostic call, which
    reads the floor every time)."""
    c = make_case(40, 40, 4, seed=77)
    pid = L.plan(c["tile"], iters=60, input_f64=True)
    y = _dev(c["y"], np.float64)
    out = torch.empty((40, 40), dtype=torch.float32, device="cuda:0")
    L.reconstruct_batch([(y, pid, out)])
    no_floor = out.clone()
    L.set_energy_floor(pid, 0.02)
    L.reconstruct_batch([(y, pid, out)])
    ref, sel = L.reconstruct_diag(y, pid)
    torch.cuda.synchronize()
    assert bool((sel < 0).any())               # some window stopped early
    assert torch.equal(out, ref)
    assert not torch.equal(out, no_floor)
    L.release(pid)
