"""The allocation-free entry point, ljsde_reconstruct_noalloc, against
ljsde_reconstruct: the same persistent FP32 kernel on the same plan and
input, with its work memory in the library's static device array instead of
allocated buffers. Outputs must be equal (the FP32 bar of 0.05 grey levels
holds a fortiori), on consecutive calls whose second image is smaller than
the first, so that the array's work list is replaced between them; the small
image is also checked against the FP64 oracle."""
import numpy as np
import pytest

from oracle import ljsde_oracle as O
from synth import QUARTER, THREE_QUARTER, random_pattern, sense, synthetic_image

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FP32_TOL = 0.05


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2205_02646_amd import ljsde
    ljsde.lib()
    return ljsde


def _image(rows, cols, tile, seed, shape=THREE_QUARTER):
    _, observed = synthetic_image(rows, cols, seed=seed)
    return sense(observed, tile, shape)


@pytest.mark.parametrize("input_f64,shape", [(True, THREE_QUARTER), (False, THREE_QUARTER), (True, QUARTER)],
                         ids=["f64in", "f32in", "quarter_f64in"])
def test_noalloc_equals_reconstruct_on_consecutive_calls_second_smaller(L, input_f64, shape):
    tile = random_pattern(4, 4, seed=31)
    iters = 40
    pid = L.plan(tile, window=32, block=4, iters=iters, rho=0.7, gamma=0.5, input_f64=input_f64,
                 shape=0 if shape == THREE_QUARTER else shape)
    dt = torch.float64 if input_f64 else torch.float32
    sizes = [(192, 160), (72, 88)]  # reconstruction rows x cols; the second is smaller
    ys, refs = [], []
    for k, (r, c) in enumerate(sizes):
        y = _image(r, c, tile, seed=40 + k, shape=shape)
        yd = torch.from_numpy(y).to("cuda:0").to(dt).contiguous()
        ys.append((y, yd))
        refs.append(L.reconstruct(yd, pid))  # allocating path: also builds the size's tables
    torch.cuda.synchronize()
    outs = [torch.full_like(ref, float("nan")) for ref in refs]
    # two calls in a row, the second with the smaller input, then the first again
    for k in (0, 1, 0):
        outs[k].fill_(float("nan"))
        print(f"noalloc call: input_f64={input_f64} shape={shape:#x} size={sizes[k]}", flush=True)
        L.reconstruct_noalloc(ys[k][1], pid, outs[k])
        torch.cuda.synchronize()
        assert torch.equal(outs[k], refs[k]), float(torch.max(torch.abs(outs[k] - refs[k])))
    # the smaller image against the FP64 oracle on the same measurements
    y_small = ys[1][0] if input_f64 else ys[1][0].astype(np.float32).astype(np.float64)
    ref64 = O.reconstruct(y_small, tile, W=32, B=4, iters=iters, rho=0.7, gamma=0.5, form="RL", shape=shape)
    err = float(np.max(np.abs(outs[1].cpu().numpy().astype(np.float64) - ref64)))
    assert err <= FP32_TOL, err
    L.release(pid)


def test_noalloc_refuses_a_size_without_resident_tables(L):
    tile = random_pattern(4, 4, seed=32)
    pid = L.plan(tile, iters=10, input_f64=True)
    y = torch.zeros((20, 24), dtype=torch.float64, device="cuda:0")
    out = torch.zeros((40, 48), dtype=torch.float32, device="cuda:0")
    with pytest.raises(L.LjsdeError) as e:
        L.reconstruct_noalloc(y, pid, out)
    assert e.value.code == L.EINVAL
    assert "tables" in str(e.value)
    L.release(pid)
