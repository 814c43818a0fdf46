"""Pins of the FP64 CPU oracle against facts the paper and the mathematics fix.

Each test checks the oracle against something other than itself: an
independently written measurement operator, brute-force least squares,
closed forms, exact-recovery cases, invariances, and the table sizes printed
in the paper. A plausible slip in the oracle (a dropped quadrant, a missing
conjugate, a wrong sign of the exponent, a shifted window or block, a
transposed operand) fails at least one of them.
"""
import json
import os

import numpy as np
import pytest

from oracle import ljsde_oracle as O
from synth import make_case, random_pattern, sense

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _psi(W):
    """Fourier basis written out independently of the oracle (Sec. III)."""
    n = np.arange(W)
    e = np.exp(2j * np.pi * np.outer(n, n) / W)
    return np.einsum("as,bt->abst", e, e)


def _window_case(W, B, seed, image=None, tile=None, rows=None, cols=None):
    rng = np.random.default_rng(seed)
    rows = rows or 2 * W
    cols = cols or 2 * W
    if image is None:
        image = rng.uniform(0, 255, size=(rows, cols))
    if tile is None:
        tile = random_pattern(4, 4, seed=seed)
    y = sense(image, tile)
    return image, tile, y


# --------------------------------------------------------------------------
# eq. (1): two independent measurement operators must agree
# --------------------------------------------------------------------------

@pytest.mark.parametrize("shape,tshape", [((8, 8), (4, 4)), ((12, 16), (2, 3)), ((16, 8), (8, 4))])
def test_sensor_readout_matches_dense_measurement_matrix(shape, tshape):
    rng = np.random.default_rng(1)
    f = rng.normal(size=shape)
    tile = rng.integers(0, 4, size=tshape).astype(np.uint8)
    np.testing.assert_allclose(sense(f, tile), O.measure_dense(f, tile), rtol=0, atol=1e-12)


def test_constant_image_reads_three_quadrants():
    tile = random_pattern(4, 4, seed=0)
    y = sense(np.full((16, 16), 7.0), tile)
    assert np.all(y == 21.0)


def test_local_operator_reproduces_global_measurements():
    """A^local applied to the image under the window equals the global
    read-out of the window's sensor pixels (window origin and offset)."""
    W, B = 32, 4
    image, tile, y = _window_case(W, B, seed=2, rows=96, cols=80)
    off = O.central_offset(W, B)
    for bi, bj in [(10, 8), (9, 7), (12, 11)]:
        y_loc, codes, valid = O.local_window(y, tile, bi, bj, W, B)
        assert valid.all()
        A = O.local_measurement_operator(codes, valid, W)
        r0, c0 = B * bi - off, B * bj - off
        fw = image[r0:r0 + W, c0:c0 + W]
        np.testing.assert_allclose(np.tensordot(A, fw, axes=([1, 2], [0, 1])), y_loc, atol=1e-9)
        assert np.all(A.reshape(A.shape[0], -1).sum(axis=1) == 3)


def test_border_window_drops_absent_measurements():
    W, B = 32, 4
    _, tile, y = _window_case(W, B, seed=3)
    y_loc, codes, valid = O.local_window(y, tile, 0, 0, W, B)
    # window of block (0, 0) starts 7 sensor pixels above/left of the image
    assert valid.sum() == 9 * 9 and not valid[:7].any() and not valid[:, :7].any()
    A = O.local_measurement_operator(codes, valid, W)
    rows = A.reshape(A.shape[0], -1).sum(axis=1)
    assert np.all(rows[~valid.reshape(-1)] == 0) and np.all(y_loc[~valid.reshape(-1)] == 0)


# --------------------------------------------------------------------------
# eqs. (9)-(11), (16): brute-force weighted least squares on tiny windows
# --------------------------------------------------------------------------

@pytest.mark.parametrize("W,B,q_mode", [(8, 4, "fsr"), (8, 4, "ones"), (16, 4, "fsr")])
def test_selection_and_step_match_bruteforce_least_squares(W, B, q_mode):
    rng = np.random.default_rng(W)
    tile = rng.integers(0, 4, size=(W // 2, W // 2)).astype(np.uint8)
    codes = tile.astype(np.int64)
    valid = np.ones_like(codes, dtype=bool)
    valid[0, :2] = False                     # a few absent measurements
    f_win = rng.uniform(0, 255, size=(W, W))
    A = O.local_measurement_operator(codes, valid, W)
    y_loc = np.tensordot(A, f_win, axes=([1, 2], [0, 1]))
    w = O.spatial_weights(W, 0.7) * valid.reshape(-1)
    q = O.frequency_weights(W, q_mode)
    Psi = _psi(W)
    a_ind = np.einsum("mab,abst->mst", A, Psi).reshape(A.shape[0], W * W)
    a = O.basis_responses(A, O.fourier_basis(W))
    gamma = 0.5
    sw = np.sqrt(w)
    for nu in range(6):
        tr = O.ljsde_window(y_loc, a, w, q, nu + 1, gamma)
        prev = O.ljsde_window(y_loc, a, w, q, nu, gamma)
        # residual of eq. (4) from the coefficients, evaluated in the pixel domain
        f_hat = np.einsum("abst,st->ab", Psi, prev.coeffs.reshape(W, W))
        r = y_loc - np.tensordot(A, f_hat, axes=([1, 2], [0, 1]))
        E = np.sum(w * np.abs(r) ** 2)
        gains = np.zeros(W * W)
        steps = np.zeros(W * W, dtype=complex)
        for k in range(W * W):
            col = (sw * a_ind[:, k])[:, None]
            if np.allclose(col, 0):
                continue
            d, *_ = np.linalg.lstsq(col, sw * r, rcond=None)
            steps[k] = d[0]
            gains[k] = E - np.sum(w * np.abs(r - d[0] * a_ind[:, k]) ** 2)
        k = tr.picks[-1]
        score = q * gains
        # the pick attains the brute-force maximum; any other frequency within
        # rounding of it is its conjugate partner (an exact tie for a real A)
        near = np.flatnonzero(score >= score.max() * (1 - 1e-10))
        assert k in near
        assert {_canon(int(j), W) for j in near} == {_canon(k, W)}
        np.testing.assert_allclose(tr.r_pick[-1] / tr.d_pick[-1], steps[k], rtol=1e-10)
        np.testing.assert_allclose(abs(tr.r_pick[-1]) ** 2 / tr.d_pick[-1], gains[k], rtol=1e-9)
        dc = tr.coeffs - prev.coeffs
        np.testing.assert_allclose(dc[k], gamma * steps[k], rtol=1e-10)
        assert np.count_nonzero(np.abs(dc) > 0) == 1


# --------------------------------------------------------------------------
# eqs. (7), (8), (15), (16): energy bookkeeping
# --------------------------------------------------------------------------

@pytest.mark.parametrize("gamma", [0.5, 1.0, 1.5])
def test_energy_follows_closed_form_and_decreases(gamma):
    W, B = 16, 4
    image, tile, y = _window_case(W, B, seed=5)
    y_loc, codes, valid = O.local_window(y, tile, 5, 6, W, B)
    A = O.local_measurement_operator(codes, valid, W)
    a = O.basis_responses(A, O.fourier_basis(W))
    w = O.spatial_weights(W, 0.7)
    tr = O.ljsde_window(y_loc, a, w, O.frequency_weights(W), 40, gamma)
    E = tr.energy0
    for e, R, D in zip(tr.energy, tr.r_pick, tr.d_pick):
        # E' = E - (2 gamma - gamma^2) |R|^2 / D for r' = r - gamma (R/D) a
        E = E - (2 * gamma - gamma ** 2) * abs(R) ** 2 / D
        assert abs(e - E) <= 1e-9 * tr.energy0
    assert all(b <= a_ * (1 + 1e-12) for a_, b in zip([tr.energy0] + tr.energy, tr.energy))


@pytest.mark.parametrize("W", [8, 16, 32])
def test_spatial_weight_is_isotropic_about_the_window_centre(W):
    """eq. (8): w_m depends only on the distance to the window centre, so it
    is invariant under both mirror flips and the transpose of the window,
    decays outwards and is largest at the four central sensor pixels."""
    w = O.spatial_weights(W, 0.7).reshape(W // 2, W // 2)
    np.testing.assert_allclose(w, w[::-1, :], rtol=1e-15)
    np.testing.assert_allclose(w, w[:, ::-1], rtol=1e-15)
    np.testing.assert_allclose(w, w.T, rtol=1e-15)
    h = W // 4
    assert np.all(np.diff(w[h, h:]) < 0) and np.all(w <= w[h, h])
    # the four central sensor pixels meet at the window centre; each one's
    # centre is one high-res pixel away along each axis: d = sqrt(2)
    np.testing.assert_allclose(w[h, h], 0.7 ** np.sqrt(2.0), rtol=1e-14)


def test_aliased_basis_functions_tie_exactly_and_the_lowest_index_wins():
    """With only orientations 1 and 3 (opaque quadrant in column 1) the
    responses at sigma = 0 are orientation-independent, H(0, rho) = 2 + e^{i theta rho},
    so a(0, rho + W/2) = a(0, rho) (2 - e^{i theta rho}) / (2 + e^{i theta rho}):
    for rho = W/4 the factor has modulus 1 and the two metrics are equal. The
    tie goes to the lower frequency index, in both formulations."""
    W = 32
    rng = np.random.default_rng(18)
    codes = np.where(rng.random((W // 2, W // 2)) < 0.5, 1, 3)
    valid = np.ones_like(codes, dtype=bool)
    A = O.local_measurement_operator(codes, valid, W)
    a = O.basis_responses(A, O.fourier_basis(W))
    k1, k2 = 0 * W + W // 4, 0 * W + 3 * W // 4
    ratio = a[:, k2] / a[:, k1]
    np.testing.assert_allclose(ratio, ratio[0], rtol=1e-12)
    assert abs(abs(ratio[0]) - 1.0) < 1e-14
    eta, gam = np.mgrid[0:W, 0:W]
    f_loc = 5.0 * np.exp(2j * np.pi * gam * (3 * W // 4) / W)      # the higher-index member
    y_loc = np.tensordot(A, f_loc, axes=([1, 2], [0, 1]))
    w = O.spatial_weights(W, 0.7)
    q = O.frequency_weights(W, "ones")
    trL = O.ljsde_window(y_loc, a, w, q, 6, 0.5)
    Bm, C, D = O.rljsde_precompute(a, w)
    trR = O.rljsde_window(y_loc, Bm, C, D, q, 6, 0.5)
    for tr in (trL, trR):
        assert tr.picks == [k1] * 6
    np.testing.assert_allclose(trL.coeffs, trR.coeffs, atol=1e-12)


# --------------------------------------------------------------------------
# Exact recovery
# --------------------------------------------------------------------------

@pytest.mark.parametrize("form", ["L", "RL"])
def test_constant_image_recovers_closed_form(form):
    """f = c: the DC basis function fits r exactly, so it wins every
    iteration and f-hat = (1 - (1 - gamma)^K) c, also in border windows."""
    W, B, K, gamma, c = 16, 4, 30, 0.5, 100.0
    tile = random_pattern(4, 4, seed=4)
    y = sense(np.full((24, 32), c), tile)
    out, tr = O.reconstruct(y, tile, W=W, B=B, iters=K, gamma=gamma, form=form, traces=True)
    np.testing.assert_allclose(out, (1 - (1 - gamma) ** K) * c, rtol=1e-12)
    assert all(set(t.picks) == {0} for t in tr.values())


@pytest.mark.parametrize("W,uv", [(16, (3, 5)), (16, (11, 2)), (32, (7, 29))])
def test_single_measurement_consistent_basis_function_is_recovered(W, uv):
    """y = A (c Phi_uv) and q = 1: by Cauchy-Schwarz every pick is (u, v)
    and c-hat_uv = (1 - (1 - gamma)^K) c (eqs. (10), (15)-(17))."""
    u, v = uv
    K, gamma, c = 12, 0.5, 3.0 - 2.0j
    rng = np.random.default_rng(7)
    codes = rng.integers(0, 4, size=(W // 2, W // 2))
    valid = np.ones_like(codes, dtype=bool)
    eta, gam = np.mgrid[0:W, 0:W]
    f_loc = c * np.exp(2j * np.pi * (eta * u + gam * v) / W)
    A = O.local_measurement_operator(codes, valid, W)
    y_loc = np.tensordot(A, f_loc, axes=([1, 2], [0, 1]))
    a = O.basis_responses(A, O.fourier_basis(W))
    w = O.spatial_weights(W, 0.7)
    q = O.frequency_weights(W, "ones")
    expect = np.zeros(W * W, dtype=complex)
    expect[u * W + v] = (1 - (1 - gamma) ** K) * c
    trL = O.ljsde_window(y_loc, a, w, q, K, gamma)
    Bm, C, D = O.rljsde_precompute(a, w)
    trR = O.rljsde_window(y_loc, Bm, C, D, q, K, gamma)
    off = O.central_offset(W, 4)
    block = np.real((1 - (1 - gamma) ** K) * f_loc[off:off + 4, off:off + 4])
    for tr in (trL, trR):
        assert tr.picks == [u * W + v] * K
        np.testing.assert_allclose(tr.coeffs, expect, atol=1e-12 * abs(c))
        # eq. (18): the back-transform reproduces the central block of the model
        np.testing.assert_allclose(O.synthesize_block(tr.coeffs, W, 4), block, atol=1e-11)


# --------------------------------------------------------------------------
# RL-JSDE == L-JSDE (Sec. IV, Sec. V-A)
# --------------------------------------------------------------------------

def _canon(k, W):
    s, r = divmod(k, W)
    return min(k, ((-s) % W) * W + (-r) % W)


def test_recurrent_equals_local_formulation():
    W, B = 32, 4
    case = make_case(32, 48, 4, seed=11)
    outL, trL = O.reconstruct(case["y"], case["tile"], W=W, B=B, iters=60, form="L", traces=True)
    outR, trR = O.reconstruct(case["y"], case["tile"], W=W, B=B, iters=60, form="RL", traces=True)
    assert np.max(np.abs(outL - outR)) <= 1e-10
    for key in trL:
        assert [_canon(k, W) for k in trL[key].picks] == [_canon(k, W) for k in trR[key].picks]


def test_projection_tables_are_consistent():
    """C is Hermitian, D its real positive diagonal, and B y equals the
    first L-JSDE numerator (eqs. (12)-(14))."""
    W = 16
    rng = np.random.default_rng(9)
    codes = rng.integers(0, 4, size=(W // 2, W // 2))
    valid = np.ones_like(codes, dtype=bool)
    A = O.local_measurement_operator(codes, valid, W)
    a = O.basis_responses(A, O.fourier_basis(W))
    w = O.spatial_weights(W, 0.7)
    Bm, C, D = O.rljsde_precompute(a, w)
    np.testing.assert_allclose(C, C.conj().T, atol=1e-10)
    assert np.all(D > 0)
    y = rng.normal(size=A.shape[0])
    # DC: every sensor pixel responds with 3, so R_00 = 3 sum w y and D_00 = 9 sum w
    R = Bm.T @ y
    np.testing.assert_allclose(R[0], 3 * np.sum(w * y), rtol=1e-12)
    np.testing.assert_allclose(D[0], 9 * np.sum(w), rtol=1e-12)


# --------------------------------------------------------------------------
# Invariances
# --------------------------------------------------------------------------

def test_conjugate_tie_gives_same_real_output():
    """A is real: for a real residual R_{-u,-v} = conj(R_uv), an exact tie.
    Taking the partner conjugates the model; the real output is unchanged."""
    W, B = 16, 4
    image, tile, y = _window_case(W, B, seed=12)
    y_loc, codes, valid = O.local_window(y, tile, 5, 5, W, B)
    A = O.local_measurement_operator(codes, valid, W)
    a = O.basis_responses(A, O.fourier_basis(W))
    w = O.spatial_weights(W, 0.7)
    q = O.frequency_weights(W)
    tr = O.ljsde_window(y_loc, a, w, q, 30, 0.5)
    nu = next(i for i, k in enumerate(tr.picks) if _canon(k, W) != k or
              ((-(k // W)) % W) * W + (-(k % W)) % W != k)
    k = tr.picks[nu]
    partner = ((-(k // W)) % W) * W + (-(k % W)) % W
    alt = O.ljsde_window(y_loc, a, w, q, 30, 0.5, force={nu: partner})
    f1 = O.synthesize_block(tr.coeffs, W, B)
    f2 = O.synthesize_block(alt.coeffs, W, B)
    np.testing.assert_allclose(f1, f2, atol=1e-9)
    assert [_canon(k, W) for k in tr.picks] == [_canon(k, W) for k in alt.picks]


def test_scale_by_power_of_two_is_exact():
    W, B = 16, 4
    case = make_case(24, 24, 4, seed=13)
    o1, t1 = O.reconstruct(case["y"], case["tile"], W=W, B=B, iters=25, form="RL", traces=True)
    o2, t2 = O.reconstruct(4.0 * case["y"], case["tile"], W=W, B=B, iters=25, form="RL", traces=True)
    assert all(t1[k].picks == t2[k].picks for k in t1)
    assert np.array_equal(4.0 * o1, o2)


def test_translation_by_one_period_shifts_the_output():
    W, B = 16, 4
    case = make_case(64, 48, 4, seed=14)
    y, tile = case["y"], case["tile"]
    blocks = [(bi, bj) for bi in range(6, 10) for bj in range(4, 8)]
    o1 = O.reconstruct(y, tile, W=W, B=B, iters=20, form="RL", blocks=blocks)
    y2 = y[4:, 4:]                           # one 4-sensor-pixel period = 8 high-res px
    blocks2 = [(bi - 2, bj - 2) for bi, bj in blocks]
    o2 = O.reconstruct(y2, tile, W=W, B=B, iters=20, form="RL", blocks=blocks2)
    np.testing.assert_array_equal(o1[24:40, 16:32], o2[16:32, 8:24])


def test_uniform_pattern_aliases_with_sensor_period():
    """With one orientation everywhere the basis responses of sigma and
    sigma + W/2 differ only by a per-frequency factor, so |R|^2 / D repeats
    with period W/2 in both axes: the aliasing that a non-regular layout
    removes."""
    W = 32
    rng = np.random.default_rng(15)
    codes = np.full((W // 2, W // 2), 2)
    valid = np.ones_like(codes, dtype=bool)
    A = O.local_measurement_operator(codes, valid, W)
    a = O.basis_responses(A, O.fourier_basis(W))
    w = O.spatial_weights(W, 0.7)
    y = rng.normal(size=A.shape[0])
    R = (a.conj().T @ (w * y)).reshape(W, W)
    D = ((w[:, None] * np.abs(a) ** 2).sum(axis=0)).reshape(W, W)
    g = np.abs(R) ** 2 / D
    h = W // 2
    np.testing.assert_allclose(g[h:, :], g[:h, :], rtol=1e-9)
    np.testing.assert_allclose(g[:, h:], g[:, :h], rtol=1e-9)
    # a random pattern breaks the repetition
    codes2 = rng.integers(0, 4, size=(W // 2, W // 2))
    a2 = O.basis_responses(O.local_measurement_operator(codes2, valid, W), O.fourier_basis(W))
    R2 = (a2.conj().T @ (w * y)).reshape(W, W)
    D2 = ((w[:, None] * np.abs(a2) ** 2).sum(axis=0)).reshape(W, W)
    g2 = np.abs(R2) ** 2 / D2
    assert np.max(np.abs(g2[h:, :] - g2[:h, :])) > 1e-3 * np.max(g2)


def test_central_block_is_the_best_modelled_part_of_the_window():
    """The spatial weight concentrates the fit on the window centre, where
    the target block is kept (eq. (8), eq. (18)): on a smooth image the
    central block is modelled far better than the window's corners."""
    W, B = 32, 4
    rng = np.random.default_rng(16)
    eta, gam = np.mgrid[0:128, 0:128].astype(float)
    clean = 128 + sum(rng.uniform(0, 40) * np.sin(2 * np.pi * rng.uniform(0.02, 0.12)
                      * (eta * np.cos(t) + gam * np.sin(t)) + rng.uniform(0, 6))
                      for t in rng.uniform(0, np.pi, 8))
    tile = random_pattern(4, 4, seed=16)
    y = sense(clean, tile)
    Phi = O.fourier_basis(W).reshape(W * W, W * W)
    errs_center, errs_corner = [], []
    off = O.central_offset(W, B)
    for bi, bj in [(12, 12), (14, 17), (17, 13), (15, 15)]:
        y_loc, codes, valid = O.local_window(y, tile, bi, bj, W, B)
        A = O.local_measurement_operator(codes, valid, W)
        a = O.basis_responses(A, O.fourier_basis(W))
        w = O.spatial_weights(W, 0.7)
        tr = O.ljsde_window(y_loc, a, w, O.frequency_weights(W), 100, 0.5)
        f = np.real(Phi @ tr.coeffs).reshape(W, W)
        r0, c0 = B * bi - off, B * bj - off
        err = (f - clean[r0:r0 + W, c0:c0 + W]) ** 2
        errs_center.append(err[off:off + B, off:off + B].mean())
        errs_corner.append(np.mean([err[:B, :B].mean(), err[:B, -B:].mean(),
                                    err[-B:, :B].mean(), err[-B:, -B:].mean()]))
    assert np.mean(errs_center) * 100 < np.mean(errs_corner)


# --------------------------------------------------------------------------
# Table sizes printed in Sec. V-B
# --------------------------------------------------------------------------

def test_precomputed_table_sizes_match_the_paper():
    with open(os.path.join(GOLDEN, "memory_table.json")) as fh:
        gold = json.load(fh)
    W, B = gold["window"], gold["block"]
    n = (W // B) ** 2
    assert n == gold["n_matrices"]
    rng = np.random.default_rng(17)
    codes = rng.integers(0, 4, size=(W // 2, W // 2))
    valid = np.ones_like(codes, dtype=bool)
    A = O.local_measurement_operator(codes, valid, W)
    a = O.basis_responses(A, O.fourier_basis(W))
    Bm, C, D = O.rljsde_precompute(a, O.spatial_weights(W, 0.7))
    entry = np.dtype(np.complex64).itemsize
    mb = lambda x: round(x.size * entry / 1e6, 1)   # noqa: E731
    assert Bm.shape == (256, 1024) and C.shape == (1024, 1024) and D.shape == (1024,)
    assert round(n * mb(Bm), 1) == gold["B_MB"]
    assert round(n * mb(C), 1) == gold["C_MB"]
    assert round(n * D.size * entry / 1e6, 1) == gold["D_MB"]
    assert round(n * (mb(Bm) + mb(C)) + round(n * D.size * entry / 1e6, 1), 1) == gold["total_MB"]
