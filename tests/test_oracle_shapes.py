"""Pins of the oracle for pixel shapes other than the L of three-quarter
sampling (Sec. I: quarter sampling collects light on one quadrant per pixel;
Sec. II, eq. (1): any such layout is a measurement matrix A).

The shape is a 4-bit mask of quadrant offsets d: the pixel of code o collects
the quadrants o XOR d for the bits d of the mask (three-quarter 0b1110,
quarter 0b0001). Checked against an independently written read-out, direct
slicing, closed forms of D and of constant images, and brute-force least
squares on the quarter-sampling operator.
"""
import numpy as np
import pytest

from oracle import ljsde_oracle as O
from synth import QUARTER, THREE_QUARTER, make_case, random_pattern, sense

ALL_SHAPES = list(range(1, 16))


def _canon(k, W):
    s, r = divmod(int(k), W)
    return min(k, ((-s) % W) * W + (-r) % W)


@pytest.mark.parametrize("shape", ALL_SHAPES)
def test_readout_matches_dense_matrix_for_every_shape(shape):
    rng = np.random.default_rng(shape)
    f = rng.normal(size=(12, 16))
    tile = rng.integers(0, 4, size=(3, 4)).astype(np.uint8)
    np.testing.assert_allclose(sense(f, tile, shape), O.measure_dense(f, tile, shape), rtol=0, atol=1e-12)


@pytest.mark.parametrize("code", [0, 1, 2, 3])
def test_quarter_sampling_with_one_code_is_plain_subsampling(code):
    """Every pixel collects the same quadrant: y is every second pixel."""
    rng = np.random.default_rng(code)
    f = rng.normal(size=(16, 20))
    tile = np.full((2, 2), code, dtype=np.uint8)
    expect = f[code >> 1::2, code & 1::2]
    np.testing.assert_array_equal(sense(f, tile, QUARTER), expect)
    np.testing.assert_allclose(O.measure_dense(f, tile, QUARTER), expect, rtol=0, atol=0)


@pytest.mark.parametrize("shape", ALL_SHAPES)
def test_constant_image_reads_the_number_of_collected_quadrants(shape):
    tile = random_pattern(4, 4, seed=shape)
    y = sense(np.full((16, 16), 7.0), tile, shape)
    assert np.all(y == 7.0 * bin(shape).count("1"))


def test_full_pixel_ignores_the_codes():
    rng = np.random.default_rng(3)
    f = rng.normal(size=(8, 8))
    box = f.reshape(4, 2, 4, 2).sum(axis=(1, 3))
    for seed in range(3):
        np.testing.assert_allclose(sense(f, random_pattern(2, 2, seed=seed), 0b1111), box, atol=1e-12)


@pytest.mark.parametrize("shape", [THREE_QUARTER, QUARTER, 0b0011, 0b0101])
def test_local_operator_rows_collect_the_shape(shape):
    W = 16
    rng = np.random.default_rng(shape)
    codes = rng.integers(0, 4, size=(W // 2, W // 2))
    valid = np.ones_like(codes, dtype=bool)
    valid[0, 0] = False
    A = O.local_measurement_operator(codes, valid, W, shape)
    rows = A.reshape(A.shape[0], -1)
    assert np.all(rows.sum(axis=1)[1:] == bin(shape).count("1")) and rows[0].sum() == 0
    # pixel (i', j') of code o collects exactly the quadrants o ^ d
    for ip, jp in [(1, 2), (5, 7), (7, 0)]:
        o = int(codes[ip, jp])
        got = {(a, b) for a in (0, 1) for b in (0, 1) if A[ip * (W // 2) + jp, 2 * ip + a, 2 * jp + b] == 1}
        want = {((o ^ d) >> 1, (o ^ d) & 1) for d in range(4) if (shape >> d) & 1}
        assert got == want


def test_quarter_sampling_normaliser_is_the_total_weight():
    """One quadrant per pixel: every basis response has modulus 1, so D of
    eq. (13) is the sum of the weights of the present pixels at every
    frequency, and the diagonal of C equals D."""
    W = 16
    rng = np.random.default_rng(4)
    codes = rng.integers(0, 4, size=(W // 2, W // 2))
    valid = np.ones_like(codes, dtype=bool)
    valid[:, 0] = False
    A = O.local_measurement_operator(codes, valid, W, QUARTER)
    a = O.basis_responses(A, O.fourier_basis(W))
    w = O.spatial_weights(W, 0.7) * valid.reshape(-1)
    _, C, D = O.rljsde_precompute(a, w)
    np.testing.assert_allclose(D, np.full(W * W, w.sum()), rtol=1e-12)
    np.testing.assert_allclose(np.diag(C).real, D, rtol=1e-12)


@pytest.mark.parametrize("W,q_mode", [(8, "fsr"), (8, "ones"), (16, "fsr")])
def test_quarter_sampling_selection_and_step_match_bruteforce_least_squares(W, q_mode):
    rng = np.random.default_rng(100 + W)
    codes = rng.integers(0, 4, size=(W // 2, W // 2))
    valid = np.ones_like(codes, dtype=bool)
    valid[1, 1:3] = False
    f_win = rng.uniform(0, 255, size=(W, W))
    A = O.local_measurement_operator(codes, valid, W, QUARTER)
    y_loc = np.tensordot(A, f_win, axes=([1, 2], [0, 1]))
    w = O.spatial_weights(W, 0.7) * valid.reshape(-1)
    q = O.frequency_weights(W, q_mode)
    n = np.arange(W)
    e = np.exp(2j * np.pi * np.outer(n, n) / W)
    Psi = np.einsum("as,bt->abst", e, e)
    a_ind = np.einsum("mab,abst->mst", A, Psi).reshape(A.shape[0], W * W)
    a = O.basis_responses(A, O.fourier_basis(W))
    gamma = 0.5
    sw = np.sqrt(w)
    for nu in range(5):
        tr = O.ljsde_window(y_loc, a, w, q, nu + 1, gamma)
        prev = O.ljsde_window(y_loc, a, w, q, nu, gamma)
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
        np.testing.assert_allclose(tr.coeffs[k] - prev.coeffs[k], gamma * steps[k], rtol=1e-10)


def test_quarter_sampling_recurrent_equals_local_formulation():
    W, B = 32, 4
    case = make_case(32, 40, 4, seed=12, shape=QUARTER)
    outL, trL = O.reconstruct(case["y"], case["tile"], W=W, B=B, iters=50, form="L", traces=True,
                              shape=QUARTER)
    outR, trR = O.reconstruct(case["y"], case["tile"], W=W, B=B, iters=50, form="RL", traces=True,
                              shape=QUARTER)
    assert np.max(np.abs(outL - outR)) <= 1e-10
    for key in trL:
        assert [_canon(k, W) for k in trL[key].picks] == [_canon(k, W) for k in trR[key].picks]


def test_quarter_sampling_of_a_measurement_consistent_basis_function_is_recovered():
    """An image that is a single (complex) basis function, sampled on one
    quadrant per pixel: the first pick is that frequency (or a tied alias) and
    the model reproduces every measurement after one full step."""
    W, B = 16, 4
    rng = np.random.default_rng(7)
    codes = rng.integers(0, 4, size=(W // 2, W // 2))
    valid = np.ones_like(codes, dtype=bool)
    A = O.local_measurement_operator(codes, valid, W, QUARTER)
    a = O.basis_responses(A, O.fourier_basis(W))
    w = O.spatial_weights(W, 0.7)
    u, v = 3, 5
    n = np.arange(W)
    f = 2.5 * np.exp(2j * np.pi * (n[:, None] * u + n[None, :] * v) / W)
    y_loc = np.tensordot(A, f, axes=([1, 2], [0, 1]))
    tr = O.ljsde_window(y_loc, a, w, np.ones(W * W), 1, 1.0)
    k = tr.picks[0]
    # the pick explains the measurements exactly
    np.testing.assert_allclose(a[:, k] * tr.coeffs[k], y_loc, atol=1e-9)


def _unobserved_closed_form(shape, codes, W):
    """Frequencies at which every present pixel's response vanishes: a pixel
    of code o responds with exp(i theta (2i' sigma + 2j' rho)) times
    sum_{d in mask} exp(i theta (qa sigma + qb rho)), q = o ^ d, and that sum
    is 0 exactly where the collected quadrants pair off with opposite phases
    (sigma or rho = W/2 for side-by-side pairs; sigma -/+ rho = W/2 for the
    diagonal pairs; one of both for the full pixel)."""
    s = np.arange(W)[:, None]
    r = np.arange(W)[None, :]
    h = W // 2
    dead = np.ones((W, W), dtype=bool)
    for o in set(int(c) for c in np.unique(codes)):
        quads = sorted(o ^ d for d in range(4) if (shape >> d) & 1)
        if quads == [0, 1] or quads == [2, 3]:
            z = np.broadcast_to(r == h, (W, W))
        elif quads == [0, 2] or quads == [1, 3]:
            z = np.broadcast_to(s == h, (W, W))
        elif quads == [0, 3]:
            z = (s + r) % W == h
        elif quads == [1, 2]:
            z = (s - r) % W == h
        elif quads == [0, 1, 2, 3]:
            z = (s == h) | (r == h)
        else:
            z = np.zeros((W, W), dtype=bool)
        dead &= z
    return dead.reshape(-1)


@pytest.mark.parametrize("shape", [0b0011, 0b0101, 0b1100, 0b0110, 0b1001, 0b1111, THREE_QUARTER, QUARTER])
def test_unobserved_frequencies_are_exactly_the_closed_form_set(shape):
    """Frequencies with no trace in the measurements get metric 0 whatever
    the residual; all others keep their q |R|^2 / D."""
    W = 16
    rng = np.random.default_rng(shape + 30)
    codes = rng.integers(0, 4, size=(W // 2, W // 2))
    valid = np.ones_like(codes, dtype=bool)
    A = O.local_measurement_operator(codes, valid, W, shape)
    a = O.basis_responses(A, O.fourier_basis(W))
    w = O.spatial_weights(W, 0.7)
    D = (w[:, None] * np.abs(a) ** 2).sum(axis=0)
    R = rng.normal(size=W * W) + 1j * rng.normal(size=W * W)
    m = O._metric(np.ones(W * W), R, D)
    dead = _unobserved_closed_form(shape, codes, W)
    assert np.array_equal(m == 0, dead)
    assert np.all(D[dead] < 1e-25 * D.max()) and np.all(D[~dead] > 1e-6 * D.max())


@pytest.mark.parametrize("shape,W", [(0b0011, 8), (0b1111, 8), (0b0110, 16)])
def test_half_and_full_pixel_selection_and_step_match_bruteforce_least_squares(shape, W):
    """Pixels that integrate two quadrants, or all four: the pick is a
    maximiser of the brute-force weighted least-squares gain over all basis
    functions, and its step is the least-squares step."""
    rng = np.random.default_rng(300 + shape + W)
    codes = rng.integers(0, 4, size=(W // 2, W // 2))
    valid = np.ones_like(codes, dtype=bool)
    valid[1, 2] = False
    f_win = rng.uniform(0, 255, size=(W, W))
    A = O.local_measurement_operator(codes, valid, W, shape)
    y_loc = np.tensordot(A, f_win, axes=([1, 2], [0, 1]))
    w = O.spatial_weights(W, 0.7) * valid.reshape(-1)
    q = O.frequency_weights(W, "fsr")
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
            col = sw * a_ind[:, k]
            nrm = np.vdot(col, col).real
            if nrm <= 1e-20 * np.sum(w) * 16:  # the column of an unobserved frequency: no gain
                continue
            d = np.vdot(col, sw * r) / nrm
            steps[k] = d
            gains[k] = E - np.sum(w * np.abs(r - d * a_ind[:, k]) ** 2)
        k = tr.picks[-1]
        score = q * gains
        near = np.flatnonzero(score >= score.max() * (1 - 1e-9))
        assert k in near
        np.testing.assert_allclose(tr.r_pick[-1] / tr.d_pick[-1], steps[k], rtol=1e-9)


@pytest.mark.parametrize("shape", [0b0011, 0b1111])
def test_half_and_full_pixel_recurrent_equals_local_formulation(shape):
    W, B = 16, 4
    case = make_case(24, 32, 4, seed=14, shape=shape)
    outL, trL = O.reconstruct(case["y"], case["tile"], W=W, B=B, iters=30, form="L", traces=True, shape=shape)
    outR, trR = O.reconstruct(case["y"], case["tile"], W=W, B=B, iters=30, form="RL", traces=True, shape=shape)
    assert np.max(np.abs(outL - outR)) <= 1e-10
    for key in trL:
        assert [_canon(k, W) for k in trL[key].picks] == [_canon(k, W) for k in trR[key].picks]
