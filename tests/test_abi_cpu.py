"""Host-side tests of the C ABI (no GPU needed): exported symbols, argument
validation, class enumeration and the FP64 per-class tables, checked against
the oracle's dense B, C, D of Sec. IV."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

from oracle import ljsde_oracle as O
from paper_2205_02646_amd import ljsde
from synth import make_case, random_pattern, random_weights

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    text = open(os.path.join(ROOT, "include", "ljsde.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ljsde_\w+)\s*\(", text)))


def test_library_exports_every_declared_function():
    names = _header_functions()
    assert len(names) >= 12
    lib = ctypes.CDLL(ljsde.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert ljsde.version() >= 10000


def _no_gpu():
    import torch
    return torch.cuda.device_count() == 0


TILE = random_pattern(4, 4, seed=0)


@pytest.mark.parametrize("kwargs,code", [
    (dict(window=30), ljsde.EINVAL),            # (W - B) not divisible by 4
    (dict(window=32, block=6), ljsde.EINVAL),
    (dict(window=33), ljsde.EINVAL),
    (dict(block=0), ljsde.EINVAL),
    (dict(iters=0), ljsde.EINVAL),
    (dict(rho=0.0), ljsde.EINVAL),
    (dict(rho=1.5), ljsde.EINVAL),
    (dict(gamma=0.0), ljsde.EINVAL),
    (dict(gamma=2.0), ljsde.EINVAL),
    (dict(window=64), ljsde.EUNSUPPORTED),      # valid for the method, no kernel
    (dict(window=32, block=12), ljsde.EUNSUPPORTED),
    (dict(fp64=True, splitbf16=True), ljsde.EINVAL),
    (dict(fp64=True, state_fp32=True), ljsde.EINVAL),
    (dict(splitbf16=True, window=16), ljsde.EUNSUPPORTED),
    (dict(dense_c=True, splitbf16=True), ljsde.EINVAL),   # options of the factorised FP32 kernel
    (dict(dense_c=True, state_fp32=True), ljsde.EINVAL),
    (dict(shape=0x3), ljsde.EUNSUPPORTED),      # half pixels: dense FP64 form only
    (dict(shape=0xF), ljsde.EUNSUPPORTED),
    (dict(shape=0x6, fp64=True), ljsde.EUNSUPPORTED),
    (dict(shape=0x6), ljsde.EUNSUPPORTED),
    (dict(shape=0x4, splitbf16=True), ljsde.EUNSUPPORTED),   # a relabelled quarter sampling
    (dict(shape=ljsde.SHAPE_QUARTER, splitbf16=True), ljsde.EUNSUPPORTED),
    (dict(shape=ljsde.SHAPE_QUARTER, state_fp32=True), ljsde.EUNSUPPORTED),
])
def test_plan_validation(kwargs, code):
    with pytest.raises(ljsde.LjsdeError) as e:
        ljsde.plan(TILE, **kwargs)
    assert e.value.code == code
    assert ljsde.last_error()


def test_plan_rejects_bad_codes_and_shapes():
    bad = TILE.copy()
    bad[1, 2] = 4
    with pytest.raises(ljsde.LjsdeError) as e:
        ljsde.plan(bad)
    assert e.value.code == ljsde.EINVAL and "not in 0..3" in str(e.value)
    L = ljsde.lib()
    assert L.ljsde_plan(None, 4, 4, 32, 4, 10, 0.7, 0.5, ljsde.FP32) == ljsde.EINVAL
    pat = np.ascontiguousarray(TILE)
    ptr = pat.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
    assert L.ljsde_plan(ptr, 0, 4, 32, 4, 10, 0.7, 0.5, ljsde.FP32) == ljsde.EINVAL
    assert L.ljsde_plan(ptr, 4, 4, 32, 4, 10, 0.7, 0.5, 0) == ljsde.EINVAL              # no precision
    assert L.ljsde_plan(ptr, 4, 4, 32, 4, 10, 0.7, 0.5, 3) == ljsde.EINVAL              # both
    assert L.ljsde_plan(ptr, 4, 4, 32, 4, 10, 0.7, 0.5, 2 | 64) == ljsde.EINVAL         # unknown flag


def test_release_and_bad_ids():
    pid = ljsde.plan(TILE)
    assert ljsde.plan_info(pid) == dict(window=32, block=4, iters=100, flags=ljsde.FP32)
    ljsde.release(pid)
    for call in (lambda: ljsde.release(pid), lambda: ljsde.plan_info(pid), lambda: ljsde.class_map(pid, 8, 8),
                 lambda: ljsde.set_energy_floor(pid, 0.1), lambda: ljsde.plan_info(-3)):
        with pytest.raises(ljsde.LjsdeError) as e:
            call()
        assert e.value.code == ljsde.EBADID


def test_energy_floor_validation():
    pid = ljsde.plan(TILE)
    ljsde.set_energy_floor(pid, 0.0)
    ljsde.set_energy_floor(pid, 1e-6)
    for bad in (-0.1, 1.0, float("nan")):
        with pytest.raises(ljsde.LjsdeError) as e:
            ljsde.set_energy_floor(pid, bad)
        assert e.value.code == ljsde.EINVAL
    ljsde.release(pid)


def test_image_size_validation():
    pid = ljsde.plan(TILE, block=8)
    for rows, cols in ((0, 8), (8, -1), (6, 8), (8, 10)):   # sides must be multiples of B/2 = 4
        with pytest.raises(ljsde.LjsdeError) as e:
            ljsde.class_map(pid, rows, cols)
        assert e.value.code == ljsde.EINVAL
    assert ljsde.class_map(pid, 12, 8)[1].shape == (3 * 2,)     # 24x16 px in 8x8 blocks
    ljsde.release(pid)


@pytest.mark.skipif(not _no_gpu(), reason="checks the no-device error path")
def test_reconstruct_without_device_reports_hip_error():
    pid = ljsde.plan(TILE)
    L = ljsde.lib()
    fake = ctypes.c_void_p(0x1000)
    assert L.ljsde_reconstruct(fake, 16, 16, pid, fake, None) == ljsde.EHIP
    assert "device" in ljsde.last_error()
    assert L.ljsde_reconstruct(None, 16, 16, pid, fake, None) == ljsde.EINVAL
    assert L.ljsde_synchronize(None) == ljsde.EHIP
    ljsde.release(pid)


# --------------------------------------------------------------------------
# Classes: windows sharing a local measurement matrix (Sec. IV)
# --------------------------------------------------------------------------

def _interior_classes(period, B=4):
    P = 2 * period
    return (P // math.gcd(P, B)) ** 2


@pytest.mark.parametrize("rows,period,interior,total", [
    (512, 4, 4, 100),      # 512x512, 4x4-sensor tile
    (2048, 8, 16, 144),    # 2048x2048, 8x8-sensor tile
    (8192, 16, 64, 256),   # 8192x8192, 16x16-sensor tile (32 px, the paper's period)
    (1200, 16, 64, 256),   # the paper's 1200x1200 frame
])
def test_class_counts(rows, period, interior, total):
    pid = ljsde.plan(random_pattern(period, period, seed=1))
    n, cls = ljsde.class_map(pid, rows // 2, rows // 2)
    assert n == total
    assert _interior_classes(period) == interior
    nb = rows // 4
    grid = cls.reshape(nb, nb)
    assert len(np.unique(grid[4:-4, 4:-4])) == interior
    ljsde.release(pid)


def test_non_recurrent_pattern_gives_one_class_per_window():
    case = make_case(64, 64, None, seed=0)
    pid = ljsde.plan(case["tile"])
    n, cls = ljsde.class_map(pid, 32, 32)
    assert n == 256 and len(np.unique(cls)) == 256
    ljsde.release(pid)


@pytest.mark.parametrize("period,rows,cols,W,B", [(4, 40, 48, 32, 4), (3, 24, 36, 16, 4), (2, 32, 24, 32, 8)])
def test_class_members_share_the_oracle_local_measurement_matrix(period, rows, cols, W, B):
    tile = random_pattern(period, period + 1, seed=period)
    pid = ljsde.plan(tile, window=W, block=B)
    y = np.zeros((rows // 2, cols // 2))
    n, cls = ljsde.class_map(pid, rows // 2, cols // 2)
    nbj = cols // B
    seen = {}
    for w, c in enumerate(cls):
        bi, bj = divmod(w, nbj)
        _, codes, valid = O.local_window(y, tile, bi, bj, W, B)
        key = np.where(valid, codes, -1)
        if c in seen:
            assert np.array_equal(seen[c], key)
        else:
            seen[c] = key
    keys = {v.tobytes() for v in seen.values()}
    assert len(keys) == n == len(seen)          # distinct classes are distinct matrices
    for c, key in seen.items():
        _, _, codes = ljsde.class_tables(pid, rows // 2, cols // 2, int(c), W)
        assert np.array_equal(codes, key)
    ljsde.release(pid)


def _H(W, shape=0xE):
    """Pixel responses H_o(sigma, rho) = sum of exp(i theta (a sigma + b rho))
    over the quadrants (a, b) the pixel of code o collects (for L pixels the
    three transparent ones; for quarter sampling quadrant o alone)."""
    s = np.arange(W)
    e = np.exp(2j * np.pi * s / W)
    out = np.zeros((4, W, W), dtype=complex)
    for o in range(4):
        for a in (0, 1):
            for b in (0, 1):
                collected = (a, b) == (o >> 1, o & 1) if shape == 0x1 else (a, b) != (o >> 1, o & 1)
                if collected:
                    out[o] += (e[:, None] ** a) * (e[None, :] ** b)
    return out


def test_shape_flags_are_kept_and_default_to_three_quarter():
    p0 = ljsde.plan(TILE)
    p1 = ljsde.plan(TILE, shape=ljsde.SHAPE_QUARTER)
    p2 = ljsde.plan(TILE, shape=ljsde.SHAPE_THREE_QUARTER, fp64=True)
    assert (ljsde.plan_info(p0)["flags"] >> 8) & 15 == 0
    assert (ljsde.plan_info(p1)["flags"] >> 8) & 15 == 0x1
    assert (ljsde.plan_info(p2)["flags"] >> 8) & 15 == 0xE
    for p in (p0, p1, p2):
        ljsde.release(p)


def test_full_reduced_precision_recipe_is_a_valid_plan():
    """LJSDE_STATE_FP32 with LJSDE_DFT_SPLITBF16 (W = 32): FP32 state, updates
    and projections with the split-BF16 window DFT."""
    pid = ljsde.plan(TILE, iters=5, state_fp32=True, splitbf16=True)
    f = ljsde.plan_info(pid)["flags"]
    assert f & ljsde.STATE_FP32 and f & ljsde.DFT_SPLITBF16
    ljsde.release(pid)


def test_float64_input_flag_is_accepted_and_kept():
    """LJSDE_INPUT_F64 (FP32 plans that read double measurements) is a known
    flag of both plan constructors and is reported back; the ABI version
    names it."""
    assert ljsde.version() >= 10200
    p0 = ljsde.plan(TILE, input_f64=True)
    p1 = ljsde.plan(TILE, input_f64=True, dense_c=True)
    p2 = ljsde.plan_weights(np.ones((2, 2, 4)), fp64=False, input_f64=True)
    for p in (p0, p1, p2):
        assert ljsde.plan_info(p)["flags"] & ljsde.INPUT_F64
        assert not ljsde.plan_info(p)["flags"] & ljsde.FP64
        ljsde.release(p)


@pytest.mark.parametrize("W,bi,bj,shape", [(32, 10, 9, 0xE), (32, 0, 3, 0xE), (16, 1, 5, 0xE),
                                           (32, 10, 9, 0x1), (16, 0, 2, 0x1)])
def test_class_tables_reproduce_dense_C_and_D(W, bi, bj, shape):
    """The library's FP64 S_o and D rebuild the oracle's dense C (eq. (14))
    and D (eq. (13)) of the same local measurement matrix, for L pixels and
    for quarter sampling."""
    tile = random_pattern(4, 4, seed=3)
    rows = cols = 96
    pid = ljsde.plan(tile, window=W, block=4, shape=shape)
    n, cls = ljsde.class_map(pid, rows // 2, cols // 2)
    c = int(cls[bi * (cols // 4) + bj])
    S, D, codes = ljsde.class_tables(pid, rows // 2, cols // 2, c, W)
    y = np.zeros((rows // 2, cols // 2))
    _, ocodes, valid = O.local_window(y, tile, bi, bj, W, 4)
    A = O.local_measurement_operator(ocodes, valid, W, shape)
    a = O.basis_responses(A, O.fourier_basis(W))
    w = O.spatial_weights(W, 0.7) * valid.reshape(-1)
    Bm, C, Dref = O.rljsde_precompute(a, w)
    np.testing.assert_allclose(D, Dref, rtol=1e-12)
    Ws = W // 2
    H = _H(W, shape).reshape(4, W * W)
    S = S.reshape(Ws, Ws, 4)
    sg = np.arange(W * W) // W
    rh = np.arange(W * W) % W
    # C[f, g] = sum_o conj(H_o(f)) H_o(g) S_o((sigma_f - sigma_g) mod Ws, (rho_f - rho_g) mod Ws)
    dk = (sg[:, None] - sg[None, :]) % Ws
    dl = (rh[:, None] - rh[None, :]) % Ws
    Cf = sum(np.conj(H[o])[:, None] * H[o][None, :] * S[dk, dl, o] for o in range(4))
    np.testing.assert_allclose(Cf, C, atol=1e-11 * np.abs(C).max())
    ljsde.release(pid)


@pytest.mark.parametrize("other", [dict(shape=ljsde.SHAPE_QUARTER), dict(splitbf16=True), dict(iters=11),
                                   dict(rho=0.6)])
def test_batch_rejects_plans_that_need_another_kernel(other):
    """All plans of one batched launch run in one kernel instantiation with
    the first plan's class-independent tables, so a batch that mixes pixel
    shapes, DFT modes, iteration counts or spatial weights (rho) is refused on
    the host (before any device work)."""
    base = dict(iters=10)
    p0 = ljsde.plan(TILE, **base)
    p1 = ljsde.plan(TILE, **{**base, **other})
    buf = (ctypes.c_float * 64)()
    addr = ctypes.cast(buf, ctypes.c_void_p).value
    jobs = (ljsde.Job * 2)(ljsde.Job(addr, 4, 4, p0, addr), ljsde.Job(addr, 4, 4, p1, addr))
    st = ljsde.lib().ljsde_reconstruct_batch(jobs, 2, None)
    assert st == ljsde.EINVAL and "job 1" in ljsde.last_error()
    ljsde.release(p0)
    ljsde.release(p1)


WTILE = random_weights(3, 4, seed=5)


@pytest.mark.parametrize("kwargs,flags,code", [
    (dict(window=30), None, ljsde.EINVAL),
    (dict(iters=0), None, ljsde.EINVAL),
    (dict(gamma=2.0), None, ljsde.EINVAL),
    (dict(window=64), None, ljsde.EUNSUPPORTED),
    (dict(), ljsde.FP32, ljsde.EUNSUPPORTED),                       # dense form only
    (dict(), ljsde.FP64, ljsde.EUNSUPPORTED),                       # not the factorised form
    (dict(), ljsde.FP64 | ljsde.DENSE_C | ljsde.SHAPE(0x1), ljsde.EINVAL),  # no pixel shape
    (dict(), ljsde.FP64 | ljsde.FP32 | ljsde.DENSE_C, ljsde.EINVAL),
    (dict(), ljsde.FP64 | ljsde.DENSE_C | 0x10000, ljsde.EINVAL),
])
def test_plan_weights_validation(kwargs, flags, code):
    args = dict(window=32, block=4, iters=10, rho=0.7, gamma=0.5)
    args.update(kwargs)
    wt = np.ascontiguousarray(WTILE)
    f = (ljsde.FP64 | ljsde.DENSE_C) if flags is None else flags
    st = ljsde.lib().ljsde_plan_weights(wt.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 3, 4,
                                        args["window"], args["block"], args["iters"], args["rho"],
                                        args["gamma"], f)
    assert st == code and ljsde.last_error()


def test_plan_weights_rejects_non_finite_weights_and_null():
    wt = WTILE.copy()
    wt[1, 2, 3] = np.nan
    with pytest.raises(ljsde.LjsdeError) as e:
        ljsde.plan_weights(wt)
    assert e.value.code == ljsde.EINVAL and "not finite" in ljsde.last_error()
    st = ljsde.lib().ljsde_plan_weights(None, 3, 4, 32, 4, 10, 0.7, 0.5, ljsde.FP64 | ljsde.DENSE_C)
    assert st == ljsde.EINVAL
    # the code-pattern constructor refuses the weights marker
    pat = np.zeros(4, np.uint8)
    st = ljsde.lib().ljsde_plan(pat.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), 2, 2, 32, 4, 10, 0.7, 0.5,
                                ljsde.FP64 | ljsde.WEIGHTS)
    assert st == ljsde.EINVAL


def test_plan_weights_info_and_class_enumeration_follow_the_tile_period():
    pid = ljsde.plan_weights(WTILE, window=32, block=4, iters=7)
    info = ljsde.plan_info(pid)
    assert info["flags"] & ljsde.WEIGHTS and info["flags"] & ljsde.DENSE_C and info["iters"] == 7
    # a 3 x 4 tile has the class structure of any 3 x 4 code pattern
    ref = ljsde.plan(random_pattern(3, 4, seed=1), window=32, block=4, fp64=True, dense_c=True)
    for rows, cols in [(48, 64), (30, 44)]:
        n1, c1 = ljsde.class_map(pid, rows, cols)
        n2, c2 = ljsde.class_map(ref, rows, cols)
        assert n1 == n2 and np.array_equal(c1, c2)
    ljsde.release(pid)
    ljsde.release(ref)


@pytest.mark.parametrize("W,bi,bj", [(32, 10, 9), (32, 0, 3), (16, 1, 5), (16, 23, 0)])
def test_weights_class_tables_reproduce_dense_C_and_D(W, bi, bj):
    """For a general layout the library's ten spectra S_qq' and D rebuild the
    oracle's dense C (eq. (14)) and D (eq. (13)) of the same local measurement
    matrix: C(f, g) = sum_{q, q'} conj(e_q(f)) e_q'(g) S_qq'(f - g) with the
    quadrant responses e_q(f) = exp(i theta (a sigma + b rho)), q = 2a + b."""
    rows = cols = 96
    pid = ljsde.plan_weights(WTILE, window=W, block=4)
    n, cls = ljsde.class_map(pid, rows // 2, cols // 2)
    c = int(cls[bi * (cols // 4) + bj])
    S, D, codes = ljsde.class_tables(pid, rows // 2, cols // 2, c, W)
    assert S.shape == ((W // 2) ** 2, 10)
    y = np.zeros((rows // 2, cols // 2))
    _, wloc, valid = O.local_window(y, WTILE, bi, bj, W, 4)
    assert np.array_equal(codes >= 0, valid) and np.all(codes[valid] == 0)
    A = O.local_measurement_operator_weights(wloc, valid, W)
    a = O.basis_responses(A, O.fourier_basis(W))
    w = O.spatial_weights(W, 0.7) * valid.reshape(-1)
    _, C, Dref = O.rljsde_precompute(a, w)
    np.testing.assert_allclose(D, Dref, rtol=1e-11)
    Ws = W // 2
    pairs = [(q, r) for q in range(4) for r in range(q, 4)]
    Sq = np.zeros((4, 4, Ws, Ws), dtype=complex)
    for k, (q, r) in enumerate(pairs):
        Sq[q, r] = Sq[r, q] = S[:, k].reshape(Ws, Ws)
    sg = np.arange(W * W) // W
    rh = np.arange(W * W) % W
    eq = np.stack([np.exp(2j * np.pi * ((q >> 1) * sg + (q & 1) * rh) / W) for q in range(4)])
    dk = (sg[:, None] - sg[None, :]) % Ws
    dl = (rh[:, None] - rh[None, :]) % Ws
    Cf = sum(np.conj(eq[q])[:, None] * eq[r][None, :] * Sq[q, r][dk, dl] for q in range(4) for r in range(4))
    np.testing.assert_allclose(Cf, C, atol=1e-11 * np.abs(C).max())
    ljsde.release(pid)


@pytest.mark.parametrize("mask,kernel_shape,d", [(0x7, 0xE, 3), (0xB, 0xE, 2), (0xD, 0xE, 1),
                                                  (0x2, 0x1, 1), (0x4, 0x1, 2), (0x8, 0x1, 3)])
def test_three_and_one_quadrant_masks_are_relabelled_layouts(mask, kernel_shape, d):
    """Three collected quadrants are three-quarter sampling with the opaque
    quadrant o ^ d (d the offset outside the mask); one collected quadrant o ^ d
    is quarter sampling with that transparent quadrant: the plan's tables equal
    those of the relabelled code tile, and its D equals the oracle's D of the
    original codes under the original mask."""
    tile = random_pattern(4, 4, seed=mask)
    W, rows, cols = 32, 96, 96
    p1 = ljsde.plan(tile, window=W, block=4, fp64=True, shape=mask)
    p2 = ljsde.plan(tile ^ d, window=W, block=4, fp64=True, shape=kernel_shape)
    n1, c1 = ljsde.class_map(p1, rows // 2, cols // 2)
    n2, c2 = ljsde.class_map(p2, rows // 2, cols // 2)
    assert n1 == n2 and np.array_equal(c1, c2)
    for c in range(n1):
        t1 = ljsde.class_tables(p1, rows // 2, cols // 2, c, W)
        t2 = ljsde.class_tables(p2, rows // 2, cols // 2, c, W)
        for a, b in zip(t1, t2):
            assert np.array_equal(a, b)
    bi, bj = 10, 9
    c = int(c1[bi * (cols // 4) + bj])
    _, D, _ = ljsde.class_tables(p1, rows // 2, cols // 2, c, W)
    _, ocodes, valid = O.local_window(np.zeros((rows // 2, cols // 2)), tile, bi, bj, W, 4)
    A = O.local_measurement_operator(ocodes, valid, W, mask)
    a = O.basis_responses(A, O.fourier_basis(W))
    _, _, Dref = O.rljsde_precompute(a, O.spatial_weights(W, 0.7) * valid.reshape(-1))
    np.testing.assert_allclose(D, Dref, rtol=1e-12)
    assert (ljsde.plan_info(p1)["flags"] >> 8) & 15 == mask
    ljsde.release(p1)
    ljsde.release(p2)


@pytest.mark.parametrize("mask", [0x3, 0x5, 0x6, 0x9, 0xA, 0xC, 0xF])
def test_two_and_four_quadrant_masks_run_as_weights_plans(mask):
    """Half, diagonal and full pixels become 0/1 quadrant weights on the dense
    FP64 form: their D rebuilds the oracle's D of the same codes and mask
    (absolutely, relative to the largest D: at the unobserved frequencies both
    are rounding noise)."""
    tile = random_pattern(4, 4, seed=mask + 7)
    W, rows, cols = 16, 48, 64
    pid = ljsde.plan(tile, window=W, block=4, fp64=True, dense_c=True, shape=mask)
    info = ljsde.plan_info(pid)
    assert info["flags"] & ljsde.WEIGHTS and (info["flags"] >> 8) & 15 == mask
    n, cls = ljsde.class_map(pid, rows // 2, cols // 2)
    for bi, bj in [(0, 0), (5, 7), (11, 15)]:
        c = int(cls[bi * (cols // 4) + bj])
        S, D, codes = ljsde.class_tables(pid, rows // 2, cols // 2, c, W)
        assert S.shape[1] == 10
        _, ocodes, valid = O.local_window(np.zeros((rows // 2, cols // 2)), tile, bi, bj, W, 4)
        A = O.local_measurement_operator(ocodes, valid, W, mask)
        a = O.basis_responses(A, O.fourier_basis(W))
        _, _, Dref = O.rljsde_precompute(a, O.spatial_weights(W, 0.7) * valid.reshape(-1))
        np.testing.assert_allclose(D, Dref, rtol=0, atol=1e-12 * Dref.max())
    ljsde.release(pid)


def test_batch_refuses_plans_without_a_batched_kernel():
    """Batched launches run the FP32 persistent kernel or the dense form: FP64
    plans of the factorised form are refused on the host."""
    pid = ljsde.plan(TILE, iters=10, fp64=True)
    buf = (ctypes.c_double * 64)()
    addr = ctypes.cast(buf, ctypes.c_void_p).value
    jobs = (ljsde.Job * 1)(ljsde.Job(addr, 4, 4, pid, addr))
    st = ljsde.lib().ljsde_reconstruct_batch(jobs, 1, None)
    assert st == ljsde.EUNSUPPORTED and "FP32" in ljsde.last_error()
    ljsde.release(pid)


@pytest.mark.parametrize("other", [dict(dense_c=False), dict(dense_c=True, rho=0.6), dict(dense_c=True, iters=11),
                                   dict(dense_c=True, fp64=False), dict(dense_c=True, shape=0x1)])
def test_dense_batch_refuses_mixed_plans(other):
    """A batch whose first plan is of the dense form runs the batched dense
    kernel: every plan must be of the dense form with equal window, block,
    iterations, rho, gamma, energy floor, pixel shape and precision (checked
    on the host, before any device work)."""
    p0 = ljsde.plan(TILE, iters=10, fp64=True, dense_c=True)
    kw = dict(iters=10, fp64=True)
    kw.update(other)
    p1 = ljsde.plan(TILE, **kw)
    buf = (ctypes.c_double * 64)()
    addr = ctypes.cast(buf, ctypes.c_void_p).value
    jobs = (ljsde.Job * 2)(ljsde.Job(addr, 4, 4, p0, addr), ljsde.Job(addr, 4, 4, p1, addr))
    assert ljsde.lib().ljsde_reconstruct_batch(jobs, 2, None) == ljsde.EINVAL
    assert "job 1" in ljsde.last_error()
    ljsde.release(p0)
    ljsde.release(p1)


def test_fp32_dense_plans_are_accepted():
    """FP32 plans of the dense form (float I/O, FP64 arithmetic), for codes,
    half pixels and general layouts."""
    pids = [ljsde.plan(TILE, iters=10, dense_c=True), ljsde.plan(TILE, iters=10, dense_c=True, shape=0x3),
            ljsde.plan_weights(WTILE, iters=10, fp64=False)]
    for pid in pids:
        f = ljsde.plan_info(pid)["flags"]
        assert f & ljsde.FP32 and f & ljsde.DENSE_C
        ljsde.release(pid)


def test_empty_batch_is_refused():
    assert ljsde.lib().ljsde_reconstruct_batch(None, 0, None) == ljsde.EINVAL
    assert ljsde.lib().ljsde_autotune(None, 0, None) == ljsde.EINVAL
    assert "empty" in ljsde.last_error()


def test_noalloc_refusals_are_host_side():
    """ljsde_reconstruct_noalloc refuses, before touching a device: plans
    without the persistent FP32 kernel, images beyond its work memory, and
    sizes whose class tables are not resident yet."""
    lib = ljsde.lib()
    fake_y, fake_out = ctypes.c_void_p(4096), ctypes.c_void_p(8192)  # never dereferenced: refused first
    p64 = ljsde.plan(TILE, iters=5, fp64=True)
    pd = ljsde.plan(TILE, iters=5, fp64=False, dense_c=True)
    ps = ljsde.plan(TILE, iters=5, state_fp32=True)
    for pid in (p64, pd, ps):
        assert lib.ljsde_reconstruct_noalloc(fake_y, 16, 16, pid, fake_out, None) == ljsde.EUNSUPPORTED
    p = ljsde.plan(TILE, iters=5)
    assert lib.ljsde_reconstruct_noalloc(None, 16, 16, p, fake_out, None) == ljsde.EINVAL
    assert lib.ljsde_reconstruct_noalloc(fake_y, 15, 16, p, fake_out, None) == ljsde.EINVAL  # odd side at B = 4
    # 2100 x 2100 sensor pixels: 1050^2 target blocks > 262144 groups of 4
    assert lib.ljsde_reconstruct_noalloc(fake_y, 2100, 2100, p, fake_out, None) == ljsde.EINVAL
    assert "work memory" in ljsde.last_error()
    # no reconstruction of this size yet: no device tables
    assert lib.ljsde_reconstruct_noalloc(fake_y, 16, 16, p, fake_out, None) == ljsde.EINVAL
    assert "tables" in ljsde.last_error()
    assert lib.ljsde_reconstruct_noalloc(fake_y, 16, 16, 10 ** 6, fake_out, None) == ljsde.EBADID
    for pid in (p64, pd, ps, p):
        ljsde.release(pid)


def test_plain_l_flag_validation():
    """LJSDE_PLAIN_L: FP64 plans, or FP32 plans (float I/O, FP64 arithmetic);
    not with the dense form, the split-BF16 DFT or the all-FP32 state; it lets
    two- and four-quadrant masks and general layouts run without
    LJSDE_DENSE_C. FP32 plain L-JSDE plans are neither batched nor taken by
    the allocation-free call."""
    assert ljsde.plan(TILE, iters=5, fp64=True, plain_l=True) >= 0
    p32 = ljsde.plan(TILE, iters=5, plain_l=True)
    assert ljsde.plan_info(p32)["flags"] & ljsde.PLAIN_L
    for bad in (dict(dense_c=True), dict(splitbf16=True), dict(state_fp32=True)):
        with pytest.raises(ljsde.LjsdeError) as e:
            ljsde.plan(TILE, iters=5, plain_l=True, **bad)
        assert e.value.code == ljsde.EINVAL
    with pytest.raises(ljsde.LjsdeError) as e:
        ljsde.plan(TILE, iters=5, fp64=True, plain_l=True, dense_c=True)
    assert e.value.code == ljsde.EINVAL
    pid = ljsde.plan(TILE, iters=5, fp64=True, plain_l=True, shape=0x3)  # half pixels
    assert ljsde.plan_info(pid)["flags"] & ljsde.WEIGHTS
    assert ljsde.plan_info(pid)["flags"] & ljsde.PLAIN_L
    wt = random_weights(2, 2, seed=1)
    pw = ljsde.plan_weights(wt, iters=5, plain_l=True)
    assert ljsde.plan_info(pw)["flags"] & ljsde.PLAIN_L
    pw32 = ljsde.plan_weights(wt, iters=5, plain_l=True, fp64=False)
    assert ljsde.plan_info(pw32)["flags"] & ljsde.FP32
    # the FP32 plain L-JSDE plan has no batched or allocation-free kernel
    buf = (ctypes.c_double * 64)()
    addr = ctypes.cast(buf, ctypes.c_void_p).value
    jobs = (ljsde.Job * 1)(ljsde.Job(addr, 4, 4, p32, addr))
    assert ljsde.lib().ljsde_reconstruct_batch(jobs, 1, None) == ljsde.EUNSUPPORTED
    assert ljsde.lib().ljsde_reconstruct_noalloc(ctypes.c_void_p(addr), 4, 4, p32, ctypes.c_void_p(addr),
                                                 None) == ljsde.EUNSUPPORTED
    for q in (p32, pid, pw, pw32):
        ljsde.release(q)
