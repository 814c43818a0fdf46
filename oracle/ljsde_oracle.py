"""Plain FP64 CPU oracle for L-JSDE and RL-JSDE.

TEST INFRASTRUCTURE ONLY. Nothing on the product path may import, call or
execute this module: only the tests, the smoke check and the CPU-baseline leg
of the benchmark use it. It shares no code with the GPU library.

It follows the paper (Grosche et al., "Fast Reconstruction of Three-Quarter
Sampling Measurements Using Recurrent Local Joint Sparse Deconvolution and
Extrapolation", IEEE TCAS-II 2022) step by step, in complex128, with no
blocking, fusion or reordering beyond what the equations state:

* ``ljsde_window`` -- L-JSDE (Sec. III and Sec. IV eqs. (2), (4)-(10), (15),
  (16)): the residual r_m is kept in the measurement domain and the selection
  numerator of eq. (10) is re-evaluated as a dense matrix-vector product every
  iteration.
* ``rljsde_precompute`` / ``rljsde_window`` -- RL-JSDE (Sec. IV eqs. (11)-(17)):
  the dense projection matrix B, the four-dimensional C (stored as a
  W^2 x W^2 matrix) and D are built for a local measurement matrix, and only
  the projected residual R is updated.
* ``synthesize_block`` -- eq. (18): back-transform and the central B x B block.
* ``reconstruct`` -- the sliding-window driver (Sec. III): one model window of
  W x W high-resolution pixels per target block of B x B, step B.

Pixel shapes (Sec. I, Sec. II eq. (1)): a sensor pixel integrates some
quadrants of its 2x2 footprint. ``shape`` is a 4-bit mask of quadrant offsets
d; the pixel with code o integrates the quadrants o XOR d for the bits d of
the mask. Three-quarter sampling, the paper's layout, is ``THREE_QUARTER =
0b1110`` (all quadrants but o, so the code names the opaque quadrant); quarter
sampling (Sec. I: one transparent quadrant per pixel) is ``QUARTER = 0b0001``
(the code names the transparent quadrant). RL-JSDE applies to any such
periodically repeating layout (Sec. I). The most general layout of this
sensor family (eq. (1) with 2x2 footprints) gives every pixel of the period
tile its own weight on each quadrant: ``weights[i, j, q]`` multiplies
quadrant q = 2a + b of the footprint of the pixel at tile position (i, j);
``reconstruct(..., weights=...)`` takes such a tile instead of codes.

Readings where the paper is silent or garbled (each is listed with its reason
in the design notes of the repository):

* Phi uses the window size W as the DFT length (the printed M, N in the basis
  definition of Sec. III is read as W; the per-class table sizes of Sec. V-B,
  256 x 1024 for B and 1024 x 1024 for C at W = 32, fix this).
* A local measurement is a sensor pixel whose 2x2 footprint lies inside the
  window: (W/2)^2 of them, index m = (W/2) * i' + j'.
* The target block sits at offset (W - B)/2 inside its window; windows step by
  B; a sensor pixel outside the image is absent (zero weight, zero row of A).
* w_m = rho ** d_m, d_m the distance in high-resolution pixels from the
  sensor-pixel centre to the window centre (eq. (8) only says isotropic and
  decaying).
* q = (1 - |f~| / (sqrt(2) W / 2))^2 with the aliased frequency magnitude
  |f~| = sqrt(min(s, W-s)^2 + min(r, W-r)^2) (Sec. IV only says it prefers low
  frequencies); ``q_mode='ones'`` gives q = 1.
* One complex coefficient per iteration, as in eqs. (15)-(17); the output is
  the real part of the central block of eq. (18).
* A frequency that leaves no trace in the window's measurements (every
  response a_m(sigma, rho) is 0, so D of eqs. (10)/(13) is 0: e.g. rho = W/2
  for pixels that integrate a horizontal pair of quadrants, or sigma = W/2 or
  rho = W/2 for full pixels) has no defined step (eq. (16) divides by D). In
  FP64 its D is rounding noise, some 1e-32 of the largest D, and its metric
  would be noise divided by noise. Reading: a frequency whose D is at most
  D_REL = 1e-13 times the largest D of the same local measurement matrix is
  unobserved and gets metric 0 (never selected); D <= 0 likewise. When every
  metric is 0 the first index is the pick; if that frequency is unobserved
  (a general layout whose weights vanish on the whole window leaves every D
  at 0) its step is 0: nothing in the window constrains it, and the model
  stays as it is.
* Ties in the argmax of eqs. (10)/(11) are left open by the paper. They are
  exact, not rare: conjugate partners tie whenever the residual is real, and
  a sparse pattern can make two basis functions alias (their measurement
  responses differ by a unit-modulus constant, so their metrics are equal).
  Reading: every metric within a relative TIE_REL = 1e-10 of the maximum
  counts as maximal and the lowest sigma * W + rho among them wins, so that
  any FP64 evaluation order resolves a tie the same way.

Parity pins (tests/test_oracle_*.py): brute-force weighted least squares on
tiny windows, the closed-form energy decrease, exact recovery of a constant
image and of a single measurement-consistent basis function, RL == L,
conjugation, scale and translation invariance, the aliasing structure of a
uniform pattern, and the table sizes printed in Sec. V-B. Image quality
itself is parity unpinned: the paper prints no quality figure.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "THREE_QUARTER",
    "QUARTER",
    "central_offset",
    "window_sensor_origin",
    "local_window",
    "local_measurement_operator",
    "local_measurement_operator_weights",
    "fourier_basis",
    "spatial_weights",
    "frequency_weights",
    "basis_responses",
    "ljsde_window",
    "rljsde_precompute",
    "rljsde_window",
    "synthesize_block",
    "reconstruct",
    "measure_dense",
    "measure_dense_weights",
    "WindowTrace",
]


THREE_QUARTER = 0b1110
QUARTER = 0b0001


def _integrates(code: int, a: int, b: int, shape: int) -> bool:
    """Whether a pixel of this code integrates quadrant (row a, column b)."""
    return bool((shape >> ((2 * a + b) ^ code)) & 1)


# ----------------------------------------------------------------------------
# Geometry (Sec. III: W x W model window, central B x B target block, step B)
# ----------------------------------------------------------------------------

def _check_geometry(W: int, B: int) -> None:
    if W <= 0 or B <= 0 or W % 2 or B % 2 or (W - B) % 4 or B > W:
        raise ValueError(f"unsupported window/block {W}/{B}: need even sizes, "
                         "B <= W and (W - B) divisible by 4")


def central_offset(W: int, B: int) -> int:
    """Offset of the target block inside its model window (Sec. IV, eq. (18))."""
    return (W - B) // 2


def window_sensor_origin(bi: int, bj: int, W: int, B: int):
    """Sensor-pixel coordinates of the window's upper-left sensor pixel.

    The window's high-resolution origin is (B*bi - (W-B)/2, B*bj - (W-B)/2);
    it is even, so it falls on a sensor-pixel corner.
    """
    off = central_offset(W, B)
    r0, c0 = B * bi - off, B * bj - off
    assert r0 % 2 == 0 and c0 % 2 == 0
    return r0 // 2, c0 // 2


def local_window(y: np.ndarray, tile: np.ndarray, bi: int, bj: int, W: int, B: int):
    """Local measurements of one window.

    Returns ``(y_loc, codes, valid)``: ``y_loc[m]`` (zero where absent),
    ``codes[i', j']`` the opaque-quadrant codes and ``valid[i', j']`` whether
    the sensor pixel exists, for the (W/2) x (W/2) sensor pixels of the window.
    """
    Ws = W // 2
    Ms, Ns = y.shape
    pr, pc = tile.shape[:2]
    rs, cs = window_sensor_origin(bi, bj, W, B)
    ii = rs + np.arange(Ws)
    jj = cs + np.arange(Ws)
    valid = ((ii >= 0) & (ii < Ms))[:, None] & ((jj >= 0) & (jj < Ns))[None, :]
    codes = tile[ii[:, None] % pr, jj[None, :] % pc]
    # a code tile gives integer codes; a weight tile [pr, pc, 4] gives the
    # window's per-pixel quadrant weights [W/2, W/2, 4]
    codes = codes.astype(np.int64) if tile.ndim == 2 else codes.astype(np.float64)
    y_loc = np.zeros((Ws, Ws), dtype=np.float64)
    iv = np.clip(ii, 0, Ms - 1)
    jv = np.clip(jj, 0, Ns - 1)
    y_loc[valid] = np.asarray(y, dtype=np.float64)[iv[:, None], jv[None, :]][valid]
    return y_loc.reshape(-1), codes, valid


# ----------------------------------------------------------------------------
# Operators of Sec. II-IV
# ----------------------------------------------------------------------------

def local_measurement_operator(codes: np.ndarray, valid: np.ndarray, W: int,
                               shape: int = THREE_QUARTER) -> np.ndarray:
    """A^local[m, eta, gamma] of eq. (4): sensor pixel m = (W/2) i' + j' sums
    the quadrants of its footprint (rows 2i', 2i'+1, columns 2j', 2j'+1 of the
    window) that its pixel shape integrates (the three transparent ones for
    three-quarter sampling); absent pixels have an all-zero row."""
    Ws = W // 2
    A = np.zeros((Ws * Ws, W, W), dtype=np.float64)
    for ip in range(Ws):
        for jp in range(Ws):
            if not valid[ip, jp]:
                continue
            o = int(codes[ip, jp])
            m = ip * Ws + jp
            for a in (0, 1):
                for b in (0, 1):
                    if _integrates(o, a, b, shape):
                        A[m, 2 * ip + a, 2 * jp + b] = 1.0
    return A


def local_measurement_operator_weights(weights: np.ndarray, valid: np.ndarray, W: int) -> np.ndarray:
    """A^local[m, eta, gamma] of eq. (4) for a general 2x2-footprint layout:
    sensor pixel m = (W/2) i' + j' weighs quadrant q = 2a + b of its footprint
    (row 2i' + a, column 2j' + b of the window) by ``weights[i', j', q]``;
    absent pixels have an all-zero row."""
    Ws = W // 2
    A = np.zeros((Ws * Ws, W, W), dtype=np.float64)
    for ip in range(Ws):
        for jp in range(Ws):
            if not valid[ip, jp]:
                continue
            m = ip * Ws + jp
            for a in (0, 1):
                for b in (0, 1):
                    A[m, 2 * ip + a, 2 * jp + b] = weights[ip, jp, 2 * a + b]
    return A


def fourier_basis(W: int) -> np.ndarray:
    """Phi[eta, gamma, sigma, rho] = exp(2 pi j (eta sigma + gamma rho) / W)
    (Sec. III, basis of eqs. (2)/(3), length W in both directions)."""
    n = np.arange(W)
    e = np.exp(2j * np.pi * np.outer(n, n) / W)  # e[eta, sigma]
    return e[:, None, :, None] * e[None, :, None, :]


def spatial_weights(W: int, rho: float) -> np.ndarray:
    """w_m of eq. (8): rho ** (distance from sensor-pixel centre to window centre)."""
    Ws = W // 2
    c = (W - 1) / 2.0
    ip, jp = np.meshgrid(np.arange(Ws), np.arange(Ws), indexing="ij")
    d = np.sqrt((2 * ip + 0.5 - c) ** 2 + (2 * jp + 0.5 - c) ** 2)
    return (rho ** d).reshape(-1)


def frequency_weights(W: int, mode: str = "fsr") -> np.ndarray:
    """q[sigma, rho] of eq. (10)/(11), flattened in sigma * W + rho order."""
    if mode == "ones":
        return np.ones(W * W)
    if mode != "fsr":
        raise ValueError(mode)
    s = np.arange(W)
    st = np.minimum(s, W - s).astype(np.float64)
    mag = np.sqrt(st[:, None] ** 2 + st[None, :] ** 2)
    return ((1.0 - mag / (np.sqrt(2.0) * W / 2.0)) ** 2).reshape(-1)


def basis_responses(A: np.ndarray, Phi: np.ndarray) -> np.ndarray:
    """a[m, sigma*W + rho] = sum_{eta, gamma} A[m, eta, gamma] Phi[eta, gamma, sigma, rho]:
    the measurement of one basis function (the inner sums of eqs. (7), (10))."""
    L = A.shape[0]
    W = A.shape[1]
    return A.reshape(L, W * W) @ Phi.reshape(W * W, W * W)


# ----------------------------------------------------------------------------
# L-JSDE (eq. (10)) and RL-JSDE (eqs. (11)-(17)) for one window
# ----------------------------------------------------------------------------

@dataclass
class WindowTrace:
    coeffs: np.ndarray                       # c-hat[sigma*W + rho], complex128
    picks: list = field(default_factory=list)       # selected sigma*W + rho
    energy: list = field(default_factory=list)      # E_w after each iteration (L-JSDE only)
    r_pick: list = field(default_factory=list)      # R_uv at selection
    d_pick: list = field(default_factory=list)      # D_uv at selection
    gap: list = field(default_factory=list)         # (best - second) / best metric
    energy0: float = 0.0


TIE_REL = 1e-10
D_REL = 1e-13


def _select(metric: np.ndarray):
    best = metric.max()
    # lowest sigma*W + rho among the metrics tied (within TIE_REL) with the maximum
    k = int(np.flatnonzero(metric >= best * (1.0 - TIE_REL))[0]) if best > 0 else 0
    if metric.size > 1 and best > 0:
        second = np.partition(metric, -2)[-2]
        gap = (best - second) / best
    else:
        gap = 0.0
    return k, gap


def _observed(D):
    # frequencies with a defined step: D > 0 and above D_REL of the largest D
    return (D > 0) & (D > D_REL * D.max())


def _metric(q, R, D):
    # q |R|^2 / D of eqs. (10)/(11); unobserved frequencies get 0
    out = np.zeros(D.shape)
    pos = _observed(D)
    out[pos] = q[pos] * np.abs(R[pos]) ** 2 / D[pos]
    return out


def _step(R, D, obs, k):
    # delta of eq. (16); an unobserved frequency takes no step
    return R[k] / D[k] if obs[k] else 0.0


def ljsde_window(y_loc, a, w, q, iters: int, gamma: float, force=None) -> WindowTrace:
    """L-JSDE on one window (O(W^4) per iteration).

    ``a`` are the basis responses (``basis_responses``), ``w`` the spatial
    weights (zero for absent measurements). The residual r starts as the
    local measurements (model initialised to zero, eq. (4)); every iteration
    evaluates eq. (10), updates one coefficient by gamma * delta (eqs. (15),
    (16)) and the residual by eq. (7). ``force`` may map an iteration index to
    a frequency index that replaces the argmax (used by invariance tests).
    """
    W2 = a.shape[1]
    D = (w[:, None] * np.abs(a) ** 2).sum(axis=0)          # denominator of eq. (10)
    r = np.asarray(y_loc, dtype=np.complex128).copy()
    tr = WindowTrace(coeffs=np.zeros(W2, dtype=np.complex128))
    tr.energy0 = float(np.sum(w * np.abs(r) ** 2))
    obs = _observed(D)
    for nu in range(iters):
        R = a.conj().T @ (w * r)                             # numerator sum of eq. (10)
        metric = _metric(q, R, D)
        k, gap = _select(metric)
        if force is not None and nu in force:
            k = force[nu]
        delta = _step(R, D, obs, k)                          # eq. (16)
        tr.coeffs[k] += gamma * delta                        # eq. (15)
        r = r - gamma * delta * a[:, k]                      # eq. (7) with the step gamma*delta
        tr.picks.append(k)
        tr.energy.append(float(np.sum(w * np.abs(r) ** 2)))  # eq. (8)
        tr.r_pick.append(R[k])
        tr.d_pick.append(D[k])
        tr.gap.append(gap)
    return tr


def rljsde_precompute(a, w):
    """Projection matrix B (eq. (12)), C (eq. (14)) and D (eq. (13)) of one
    local measurement matrix. B is returned as B[m, sigma*W + rho]; C as
    C[sigma*W + rho, u*W + v]."""
    Bm = np.conj(a) * w[:, None]
    C = Bm.T @ a
    D = np.real(np.diag(C)).copy()
    return Bm, C, D


def rljsde_window(y_loc, Bm, C, D, q, iters: int, gamma: float, force=None) -> WindowTrace:
    """RL-JSDE on one window: only the projected residual R is kept (eq. (12)
    with r = y at the start), selected by eq. (11) and updated by eq. (17)."""
    W2 = C.shape[0]
    R = Bm.T @ np.asarray(y_loc, dtype=np.complex128)        # eq. (12), iteration 0
    tr = WindowTrace(coeffs=np.zeros(W2, dtype=np.complex128))
    obs = _observed(D)
    for nu in range(iters):
        metric = _metric(q, R, D)                            # eq. (11)
        k, gap = _select(metric)
        if force is not None and nu in force:
            k = force[nu]
        delta = _step(R, D, obs, k)                          # eq. (16)
        tr.coeffs[k] += gamma * delta                        # eq. (15)
        tr.picks.append(k)
        tr.r_pick.append(R[k])
        tr.d_pick.append(D[k])
        tr.gap.append(gap)
        R = R - gamma * delta * C[:, k]                      # eq. (17)
    return tr


def synthesize_block(coeffs, W: int, B: int) -> np.ndarray:
    """eq. (18): f-hat = sum Phi c-hat on the window; the real part of the
    central B x B block is returned."""
    Phi = fourier_basis(W)
    f = Phi.reshape(W * W, W * W) @ coeffs
    off = central_offset(W, B)
    return np.real(f.reshape(W, W)[off:off + B, off:off + B])


# ----------------------------------------------------------------------------
# Sliding-window driver
# ----------------------------------------------------------------------------

class _Cache:
    def __init__(self, W, rho, form, shape=THREE_QUARTER):
        self.W = W
        self.shape = shape
        self.Phi = fourier_basis(W)
        self.w_full = spatial_weights(W, rho)
        self.form = form
        self.store = {}

    def get(self, codes, valid):
        key = (codes.tobytes(), valid.tobytes())
        hit = self.store.get(key)
        if hit is None:
            if codes.ndim == 3:
                A = local_measurement_operator_weights(codes, valid, self.W)
            else:
                A = local_measurement_operator(codes, valid, self.W, self.shape)
            a = basis_responses(A, self.Phi)
            w = self.w_full * valid.reshape(-1)
            if self.form == "RL":
                hit = (a, w) + rljsde_precompute(a, w)
            else:
                hit = (a, w)
            self.store[key] = hit
        return hit


def reconstruct(y, tile, W=32, B=4, iters=100, rho=0.7, gamma=0.5, form="L",
                q_mode="fsr", blocks=None, traces=False, shape=THREE_QUARTER, weights=None):
    """Reconstruct the 2x-resolution image from sensor read-out ``y``.

    ``tile`` is the pattern tile of quadrant codes (sensor pixel (i, j) uses
    ``tile[i % pr, j % pc]``); ``shape`` the pixel shape (module docstring).
    ``weights`` (a [pr, pc, 4] tile of per-pixel quadrant weights) replaces
    ``tile`` and ``shape`` for a general layout. ``form`` is ``"L"`` (L-JSDE) or ``"RL"``
    (RL-JSDE, per-class B, C, D cached by the content of the local measurement
    matrix). ``blocks`` restricts the work to a list of (bi, bj) target
    blocks; other output pixels are NaN. Returns the image, and with
    ``traces=True`` also a dict {(bi, bj): WindowTrace}.
    """
    _check_geometry(W, B)
    if weights is not None:
        tile = np.asarray(weights, dtype=np.float64)
        if tile.ndim != 3 or tile.shape[2] != 4:
            raise ValueError("weights must be a [rows, cols, 4] tile")
    y = np.asarray(y, dtype=np.float64)
    Ms, Ns = y.shape
    M, N = 2 * Ms, 2 * Ns
    if M % B or N % B:
        raise ValueError("image sides must be multiples of the block size")
    q = frequency_weights(W, q_mode)
    cache = _Cache(W, rho, form, shape)
    if blocks is None:
        blocks = [(bi, bj) for bi in range(M // B) for bj in range(N // B)]
    out = np.full((M, N), np.nan)
    all_traces = {}
    for bi, bj in blocks:
        y_loc, codes, valid = local_window(y, tile, bi, bj, W, B)
        if form == "RL":
            a, w, Bm, C, D = cache.get(codes, valid)
            tr = rljsde_window(y_loc, Bm, C, D, q, iters, gamma)
        elif form == "L":
            a, w = cache.get(codes, valid)
            tr = ljsde_window(y_loc, a, w, q, iters, gamma)
        else:
            raise ValueError(form)
        out[B * bi:B * bi + B, B * bj:B * bj + B] = synthesize_block(tr.coeffs, W, B)
        if traces:
            all_traces[(bi, bj)] = tr
    return (out, all_traces) if traces else out


def measure_dense_weights(f: np.ndarray, weights: np.ndarray) -> np.ndarray:
    """eq. (1) for a general layout with an explicitly built global
    measurement matrix (tiny images only): y_i = sum A_i f with the pixel at
    tile position (i % pr, j % pc) weighing quadrant q by weights[..., q]."""
    M, N = f.shape
    Ms, Ns = M // 2, N // 2
    pr, pc = weights.shape[:2]
    A = np.zeros((Ms * Ns, M, N))
    for i in range(Ms):
        for j in range(Ns):
            for a in (0, 1):
                for b in (0, 1):
                    A[i * Ns + j, 2 * i + a, 2 * j + b] = weights[i % pr, j % pc, 2 * a + b]
    return np.tensordot(A, f, axes=([1, 2], [0, 1])).reshape(Ms, Ns)


def measure_dense(f: np.ndarray, tile: np.ndarray, shape: int = THREE_QUARTER) -> np.ndarray:
    """eq. (1) with an explicitly built global measurement matrix A[i, alpha, beta]
    (for tiny images only): y_i = sum A_i f."""
    M, N = f.shape
    Ms, Ns = M // 2, N // 2
    pr, pc = tile.shape
    A = np.zeros((Ms * Ns, M, N))
    for i in range(Ms):
        for j in range(Ns):
            o = int(tile[i % pr, j % pc])
            for a in (0, 1):
                for b in (0, 1):
                    if _integrates(o, a, b, shape):
                        A[i * Ns + j, 2 * i + a, 2 * j + b] = 1.0
    return np.tensordot(A, f, axes=([1, 2], [0, 1])).reshape(Ms, Ns)
