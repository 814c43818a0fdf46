"""GPU parity on a seeded random sweep of small cases: window and block sizes,
image sides, pattern periods, iteration counts, rho, gamma, the frequency
weight and every plan type (FP64 factorised and dense, FP32 batched and dense,
general layouts, further pixel shapes in FP64 and FP32) against the FP64 CPU
oracle. FP32 plans read float64 measurements in every other case (the
oracle's own input) and float32 ones otherwise (the oracle then runs on those
values). Same bars as the other parity tests."""
import numpy as np
import pytest

from oracle import ljsde_oracle as O
from synth import make_case, random_weights, sense_weights, synthetic_image

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

KINDS = ["fp64", "dense64", "fp32", "dense32", "weights64", "mask", "mask32"]


def _draw(i):
    rng = np.random.default_rng(5000 + i)
    W = int(rng.choice([16, 32]))
    B = int(rng.choice([4, 8]))
    rows, cols = int(rng.integers(2, 7)) * 8, int(rng.integers(2, 7)) * 8
    per = int(rng.choice([2, 3, 4]))
    iters = int(rng.integers(5, 80))
    rho = round(float(rng.uniform(0.4, 1.0)), 2)
    gamma = round(float(rng.uniform(0.2, 1.8)), 2)
    q_ones = bool(rng.random() < 0.25)
    shape = [0x7, 0x2, 0x3, 0x6][(i // 7) % 4]   # "mask" cases (dense form)
    if i % 7 == 6:                                # "mask32": relabelled onto the factorised kernels
        shape = [0x7, 0x2, 0xB, 0x4][(i // 7) % 4]
    return W, B, rows, cols, per, iters, rho, gamma, q_ones, shape


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2205_02646_amd import ljsde
    ljsde.lib()
    return ljsde


@pytest.mark.parametrize("i", range(35))
def test_random_case_matches_oracle(L, i):
    kind = KINDS[i % len(KINDS)]
    W, B, rows, cols, per, iters, rho, gamma, q_ones, shape = _draw(i)
    if not kind.startswith("mask"):
        shape = 0xE
    seed = 700 + i
    wt = tile = None
    if kind == "weights64":
        wt = random_weights(per, per, seed=seed)
        _, f = synthetic_image(rows, cols, seed=seed)
        y = sense_weights(f, wt)
    else:
        c = make_case(rows, cols, per, seed=seed, shape=shape)
        y, tile = c["y"], c["tile"]
    fp32 = kind in ("fp32", "dense32", "mask32")
    f64in = not fp32 or (i // len(KINDS)) % 2 == 1
    if not f64in:
        y = y.astype(np.float32).astype(np.float64)   # the oracle runs on the float32 input
    ref, tr = O.reconstruct(y, tile, W=W, B=B, iters=iters, rho=rho, gamma=gamma, form="RL", traces=True,
                            q_mode="ones" if q_ones else "fsr", shape=shape, weights=wt)
    kw = dict(window=W, block=B, iters=iters, rho=rho, gamma=gamma, q_ones=q_ones)
    if kind == "weights64":
        pid = L.plan_weights(wt, **kw)
    elif kind == "mask":
        pid = L.plan(tile, fp64=True, dense_c=True, shape=shape, **kw)
    elif kind == "mask32":
        pid = L.plan(tile, shape=shape, input_f64=f64in, **kw)
    else:
        pid = L.plan(tile, fp64=not fp32, dense_c=kind.startswith("dense"), input_f64=fp32 and f64in, **kw)
    dt = np.float64 if f64in else np.float32
    out, sel = L.reconstruct_diag(torch.from_numpy(np.ascontiguousarray(y, dtype=dt)).to("cuda:0"), pid)
    out = out.cpu().numpy().astype(np.float64)
    sel = sel.cpu().numpy()
    err = float(np.max(np.abs(out - ref)))
    print(f"case {i} {kind} W={W} B={B} {rows}x{cols} period {per} iters {iters} rho {rho} gamma {gamma} "
          f"q {'ones' if q_ones else 'fsr'} shape 0x{shape:x} {'float64' if f64in else 'float32'} input: "
          f"max-abs {err:.2e}", flush=True)
    assert err <= (0.05 if fp32 else 1e-9)
    nbj = out.shape[1] // B
    for w in range(sel.shape[0]):
        assert list(sel[w]) == tr[divmod(w, nbj)].picks, w
    if kind in ("fp32", "mask32"):   # the batched launch gives the same image
        out_b = L.reconstruct(torch.from_numpy(np.ascontiguousarray(y, dtype=dt)).to("cuda:0"), pid)
        assert np.array_equal(out_b.cpu().numpy().astype(np.float64), out)
    L.release(pid)
