"""Pins of the oracle for general layouts of the 2x2-footprint sensor family
(Sec. II, eq. (1): each measurement is a weighted sum over its pixel's four
high-resolution quadrants; Sec. I: RL-JSDE covers any periodically repeating
layout). A tile of per-pixel quadrant weights replaces the codes.

Checked against an independently written read-out, the code/shape operator
for 0/1 weights (whole reconstructions must agree bitwise), brute-force least
squares on random weights, RL == L, and exact power-of-two scaling of weights
and measurements.
"""
import numpy as np
import pytest

from oracle import ljsde_oracle as O
from synth import (QUARTER, THREE_QUARTER, make_case, random_pattern, random_weights, sense, sense_weights,
                   shape_weights, synthetic_image)


def _canon(k, W):
    s, r = divmod(int(k), W)
    return min(k, ((-s) % W) * W + (-r) % W)


@pytest.mark.parametrize("tshape", [(3, 4), (2, 2), (5, 1)])
def test_weighted_readout_matches_dense_matrix(tshape):
    rng = np.random.default_rng(sum(tshape))
    f = rng.normal(size=(12, 16))
    wt = rng.uniform(-1, 2, size=tshape + (4,))
    np.testing.assert_allclose(sense_weights(f, wt), O.measure_dense_weights(f, wt), rtol=0, atol=1e-12)


@pytest.mark.parametrize("shape", [THREE_QUARTER, QUARTER, 0b0110])
def test_zero_one_weights_reproduce_the_code_layout(shape):
    rng = np.random.default_rng(shape)
    f = rng.normal(size=(16, 20))
    tile = rng.integers(0, 4, size=(4, 5)).astype(np.uint8)
    np.testing.assert_allclose(sense_weights(f, shape_weights(tile, shape)), sense(f, tile, shape),
                               rtol=0, atol=1e-12)
    W = 16
    codes = rng.integers(0, 4, size=(W // 2, W // 2))
    valid = np.ones_like(codes, dtype=bool)
    valid[2, :3] = False
    A1 = O.local_measurement_operator(codes, valid, W, shape)
    A2 = O.local_measurement_operator_weights(shape_weights(codes, shape), valid, W)
    np.testing.assert_array_equal(A1, A2)


def test_reconstruction_from_zero_one_weights_equals_the_code_path():
    case = make_case(32, 40, 4, seed=21)
    wt = shape_weights(case["tile"], THREE_QUARTER)
    for form in ("L", "RL"):
        a = O.reconstruct(case["y"], case["tile"], W=16, B=4, iters=30, form=form)
        b = O.reconstruct(case["y"], None, W=16, B=4, iters=30, form=form, weights=wt)
        np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("W,q_mode", [(8, "fsr"), (16, "ones")])
def test_general_layout_selection_and_step_match_bruteforce_least_squares(W, q_mode):
    rng = np.random.default_rng(200 + W)
    weights = rng.uniform(0, 1, size=(W // 2, W // 2, 4))
    valid = np.ones(weights.shape[:2], dtype=bool)
    valid[0, 1] = False
    f_win = rng.uniform(0, 255, size=(W, W))
    A = O.local_measurement_operator_weights(weights, valid, W)
    y_loc = np.tensordot(A, f_win, axes=([1, 2], [0, 1]))
    w = O.spatial_weights(W, 0.7) * valid.reshape(-1)
    q = O.frequency_weights(W, q_mode)
    n = np.arange(W)
    e = np.exp(2j * np.pi * np.outer(n, n) / W)
    Psi = np.einsum("as,bt->abst", e, e)
    a_ind = np.einsum("mab,abst->mst", A, Psi).reshape(A.shape[0], W * W)
    a = O.basis_responses(A, O.fourier_basis(W))
    sw = np.sqrt(w)
    for nu in range(4):
        tr = O.ljsde_window(y_loc, a, w, q, nu + 1, 0.5)
        prev = O.ljsde_window(y_loc, a, w, q, nu, 0.5)
        f_hat = np.einsum("abst,st->ab", Psi, prev.coeffs.reshape(W, W))
        r = y_loc - np.tensordot(A, f_hat, axes=([1, 2], [0, 1]))
        E = np.sum(w * np.abs(r) ** 2)
        gains = np.zeros(W * W)
        steps = np.zeros(W * W, dtype=complex)
        for k in range(W * W):
            col = (sw * a_ind[:, k])[:, None]
            d, *_ = np.linalg.lstsq(col, sw * r, rcond=None)
            steps[k] = d[0]
            gains[k] = E - np.sum(w * np.abs(r - d[0] * a_ind[:, k]) ** 2)
        k = tr.picks[-1]
        score = q * gains
        near = np.flatnonzero(score >= score.max() * (1 - 1e-10))
        assert k in near and k == near.min()
        np.testing.assert_allclose(tr.r_pick[-1] / tr.d_pick[-1], steps[k], rtol=1e-10)


def test_general_layout_recurrent_equals_local_formulation():
    W, B = 32, 4
    _, f = synthetic_image(32, 40, seed=13)
    wt = random_weights(4, 4, seed=13)
    y = sense_weights(f, wt)
    outL, trL = O.reconstruct(y, None, W=W, B=B, iters=40, form="L", traces=True, weights=wt)
    outR, trR = O.reconstruct(y, None, W=W, B=B, iters=40, form="RL", traces=True, weights=wt)
    assert np.max(np.abs(outL - outR)) <= 1e-10
    for key in trL:
        assert [_canon(k, W) for k in trL[key].picks] == [_canon(k, W) for k in trR[key].picks]


def test_scaling_weights_and_measurements_by_two_is_exact():
    """A' = 2A and y' = 2y give R' = 4R and D' = 4D, so every step, pick and
    output is unchanged (bitwise, powers of two)."""
    _, f = synthetic_image(24, 32, seed=14)
    wt = random_weights(3, 4, seed=14)
    y = sense_weights(f, wt)
    a = O.reconstruct(y, None, W=16, B=4, iters=25, form="RL", weights=wt)
    b = O.reconstruct(2.0 * y, None, W=16, B=4, iters=25, form="RL", weights=2.0 * wt)
    np.testing.assert_array_equal(a, b)


def test_window_without_weighted_measurements_takes_no_step():
    """A general layout whose quadrant weights vanish on a whole window leaves
    every response a_m(sigma, rho) of that window at 0: the weighted least
    squares of eq. (9) has no term, every step fits equally, and its
    minimum-norm solution (numpy.linalg.lstsq) is 0. The oracle keeps that
    window's model at 0 (first index picked, zero step), in both forms, and
    stays finite elsewhere."""
    W, B = 16, 4
    # W = 16, B = 4: window sensor rows start at 2 bi - 3, eight rows; with a
    # 16-row period whose rows 0..8 carry no weight, blocks bi = 2 (mod 8)
    # see no weighted measurement
    wt = random_weights(16, 4, seed=15)
    wt[:9] = 0.0
    _, f = synthetic_image(64, 32, seed=15)
    y = sense_weights(f, wt)
    nbj = 32 // B
    for form in ("L", "RL"):
        out, tr = O.reconstruct(y, None, W=W, B=B, iters=20, form=form, traces=True, weights=wt)
        assert np.all(np.isfinite(out))
        for bi in (2, 10):
            assert np.all(out[B * bi:B * bi + B] == 0.0)
            for bj in range(nbj):
                assert tr[(bi, bj)].picks == [0] * 20
        assert np.any(out[B * 4:B * 4 + B] != 0.0)
    # the minimum-norm least-squares step of eq. (9) on such a window
    y_loc, codes, valid = O.local_window(y, wt, 2, 3, W, B)
    a = O.basis_responses(O.local_measurement_operator_weights(codes, valid, W), O.fourier_basis(W))
    assert not np.any(a)
    sw = np.sqrt(O.spatial_weights(W, 0.7) * valid.reshape(-1))
    for k in (0, 5, 77):
        step = np.linalg.lstsq((sw * a[:, k])[:, None], sw * y_loc.astype(complex), rcond=None)[0]
        assert step[0] == 0.0
