"""Seeded synthetic inputs for three-quarter-sampling reconstruction.

This module is shared by the CPU oracle, the tests and the benchmark. It holds
no reconstruction arithmetic: it only draws test images, opaque-quadrant
patterns and the sensor read-out that a three-quarter-sampling sensor would
produce from them (Sec. II, eq. (1): each low-resolution pixel integrates the
three transparent quadrants of its 2x2 high-resolution footprint).

Conventions
-----------
* Images are indexed ``[row, col]`` with the origin in the upper-left corner.
  Sizes quoted as ``WxH`` are width x height, i.e. ``H`` rows.
* A pattern is a ``uint8`` tile of quadrant codes ``o = 2*a + b``
  (``a`` = row offset, ``b`` = column offset inside the 2x2 footprint). Sensor
  pixel ``(i, j)`` uses ``tile[i % pr, j % pc]``.
* A pixel shape is a 4-bit mask of quadrant offsets ``d``: the pixel of code
  ``o`` collects light on the quadrants ``o ^ d`` for the bits ``d`` of the
  mask. ``THREE_QUARTER = 0b1110`` (all quadrants but ``o``: the code names
  the opaque quadrant) is the default; ``QUARTER = 0b0001`` (only ``o``: the
  code names the transparent quadrant).
* Grey range is 0..255.

Workload recipe (stand-in for the paper's natural-image test set, which is not
available here): 128 grey base, plus 8 sinusoids with random orientation,
amplitude U(0, 40), spatial frequency U(0.02, 0.45) cycles/px and phase, plus
4 random polygons (3-6 vertices, ordered by angle around their centroid) with
an additive constant U(-64, 64); clipped to [0, 255]. Optional Gaussian noise
is added after clipping and not re-clipped.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "synthetic_image",
    "random_pattern",
    "sense",
    "make_case",
    "CONFIGS",
    "batch_cases",
    "THREE_QUARTER",
    "QUARTER",
    "sense_weights",
    "random_weights",
    "shape_weights",
]

THREE_QUARTER = 0b1110
QUARTER = 0b0001


def _streams(seed: int):
    ss = np.random.SeedSequence(seed)
    return [np.random.default_rng(s) for s in ss.spawn(4)]


def _fill_polygon(rows, cols, verts, r0=0, c0=0):
    """Boolean mask of pixel centres inside a simple polygon (even-odd rule),
    evaluated on the pixels [r0, r0 + rows) x [c0, c0 + cols) of the image.

    Scanline form: on the row through py = row + 0.5 a pixel centre px is
    inside when an odd number of edge crossings x satisfies x <= px (edges are
    half-open in y). With the crossings sorted, that is
    px in [x1, x2) u [x3, x4) u ..., i.e. columns ceil(xa - 1/2) .. ceil(xb - 1/2) - 1.
    """
    py = np.arange(r0, r0 + rows) + 0.5
    n = len(verts)
    xs = np.full((rows, n), np.inf)
    for k in range(n):
        y0, x0 = verts[k]
        y1, x1 = verts[(k + 1) % n]
        if y0 == y1:
            continue
        cond = (py >= min(y0, y1)) & (py < max(y0, y1))
        xs[cond, k] = x0 + (py[cond] - y0) * (x1 - x0) / (y1 - y0)
    xs.sort(axis=1)
    diff = np.zeros((rows, cols + 1), dtype=np.int16)
    ridx = np.arange(rows)
    for k in range(0, n - 1, 2):
        xa, xb = xs[:, k], xs[:, k + 1]
        ok = np.isfinite(xa) & np.isfinite(xb)
        start = np.clip(np.ceil(xa[ok] - 0.5) - c0, 0, cols).astype(np.intp)
        end = np.clip(np.ceil(xb[ok] - 0.5) - c0, 0, cols).astype(np.intp)
        np.add.at(diff, (ridx[ok], start), 1)
        np.add.at(diff, (ridx[ok], end), -1)
    return np.cumsum(diff[:, :cols], axis=1) > 0


def synthetic_image(rows: int, cols: int, seed: int = 0, noise_sigma: float = 0.0, region=None):
    """Return ``(clean, observed)`` float64 images of shape (rows, cols).

    ``observed`` equals ``clean`` plus N(0, noise_sigma^2) noise (no re-clip).
    ``region = (r0, r1, c0, c1)`` evaluates only that part of the full image
    (same values as the corresponding slice of the full image; the noise of a
    region is drawn for the region alone, so use it with noise_sigma = 0).
    """
    g_img, g_poly, _, g_noise = _streams(seed)
    r0, r1, c0, c1 = (0, rows, 0, cols) if region is None else region
    eta = np.arange(r0, r1, dtype=np.float64)
    gam = np.arange(c0, c1, dtype=np.float64)
    f = np.full((r1 - r0, c1 - c0), 128.0)
    for _ in range(8):
        amp = g_img.uniform(0.0, 40.0)
        th = g_img.uniform(0.0, np.pi)
        phi = g_img.uniform(0.02, 0.45)
        psi = g_img.uniform(0.0, 2.0 * np.pi)
        a = 2.0 * np.pi * phi * np.cos(th) * eta
        b = 2.0 * np.pi * phi * np.sin(th) * gam + psi
        # sin(a + b) = sin(a) cos(b) + cos(a) sin(b)
        f += amp * (np.sin(a)[:, None] * np.cos(b)[None, :] + np.cos(a)[:, None] * np.sin(b)[None, :])
    for _ in range(4):
        nv = int(g_poly.integers(3, 7))
        vy = g_poly.uniform(0.0, rows, size=nv)
        vx = g_poly.uniform(0.0, cols, size=nv)
        cy, cx = vy.mean(), vx.mean()
        order = np.argsort(np.arctan2(vy - cy, vx - cx))
        verts = np.stack([vy[order], vx[order]], axis=1)
        val = g_poly.uniform(-64.0, 64.0)
        f += val * _fill_polygon(r1 - r0, c1 - c0, verts, r0, c0)
    clean = np.clip(f, 0.0, 255.0)
    observed = clean
    if noise_sigma > 0.0:
        observed = clean + g_noise.normal(0.0, noise_sigma, size=clean.shape)
    return clean, observed


def random_pattern(pat_rows: int, pat_cols: int, seed: int = 0) -> np.ndarray:
    """i.i.d. uniform opaque-quadrant codes in {0,1,2,3} (uint8 tile)."""
    _, _, g_pat, _ = _streams(seed)
    return g_pat.integers(0, 4, size=(pat_rows, pat_cols)).astype(np.uint8)


def sense(image: np.ndarray, tile: np.ndarray, shape: int = THREE_QUARTER) -> np.ndarray:
    """Sensor read-out of a high-resolution image.

    Each sensor pixel ``(i, j)`` returns the sum of the quadrants of
    ``image[2i:2i+2, 2j:2j+2]`` that its shape collects: for three-quarter
    sampling the whole 2x2 sum minus the opaque quadrant selected by the tile
    code. Works for float and complex images; the result has shape
    ``(rows/2, cols/2)``.
    """
    rows, cols = image.shape
    if rows % 2 or cols % 2:
        raise ValueError("image sides must be even")
    sr, sc = rows // 2, cols // 2
    quads = image.reshape(sr, 2, sc, 2).transpose(0, 2, 1, 3)  # [i, j, a, b]
    pr, pc = tile.shape
    codes = tile[np.arange(sr)[:, None] % pr, np.arange(sc)[None, :] % pc]
    ii, jj = np.meshgrid(np.arange(sr), np.arange(sc), indexing="ij")
    out = np.zeros((sr, sc), dtype=np.result_type(image.dtype, np.float64))
    for d in range(4):
        if (shape >> d) & 1:
            q = codes.astype(np.intp) ^ d
            out = out + quads[ii, jj, q >> 1, q & 1]
    return out


def sense_weights(image: np.ndarray, weights: np.ndarray) -> np.ndarray:
    """Read-out of a general 2x2-footprint sensor: the pixel at tile position
    (i % pr, j % pc) weighs quadrant q = 2a + b of ``image[2i:2i+2, 2j:2j+2]``
    by ``weights[i % pr, j % pc, q]``."""
    rows, cols = image.shape
    sr, sc = rows // 2, cols // 2
    pr, pc = weights.shape[:2]
    quads = image.reshape(sr, 2, sc, 2).transpose(0, 2, 1, 3).reshape(sr, sc, 4)
    wt = weights[np.arange(sr)[:, None] % pr, np.arange(sc)[None, :] % pc]
    return np.einsum("ijq,ijq->ij", wt, quads)


def random_weights(pat_rows: int, pat_cols: int, seed: int = 0) -> np.ndarray:
    """A general layout: every tile pixel weighs each quadrant by U(0, 1)
    (partially transparent masks), with one quadrant of every pixel at most
    0.1 (mostly opaque)."""
    g = np.random.default_rng(np.random.SeedSequence(seed).spawn(6)[5])
    w = g.uniform(0.0, 1.0, size=(pat_rows, pat_cols, 4))
    dark = g.integers(0, 4, size=(pat_rows, pat_cols))
    np.put_along_axis(w, dark[..., None], g.uniform(0.0, 0.1, size=(pat_rows, pat_cols, 1)), axis=2)
    return w


def shape_weights(tile: np.ndarray, shape: int = THREE_QUARTER) -> np.ndarray:
    """The 0/1 weight tile of a code tile under a pixel shape."""
    q = np.arange(4)
    return (((shape >> (q[None, None, :] ^ tile[..., None].astype(np.int64))) & 1)).astype(np.float64)


# Workloads. ``pattern`` is the tile size in sensor pixels; None means the
# tile covers the whole sensor (a non-recurrent pattern).
CONFIGS = {
    0: dict(rows=64, cols=64, pattern=None, iters=100, noise=0.0),
    1: dict(rows=512, cols=512, pattern=4, iters=100, noise=0.0),
    2: dict(rows=2048, cols=2048, pattern=8, iters=250, noise=2.0),
    4: dict(rows=8192, cols=8192, pattern=16, iters=250, noise=0.0),
    # the paper's own shape: 1200x1200 grey, pattern period 32 high-res px
    "P": dict(rows=1200, cols=1200, pattern=16, iters=100, noise=0.0),
}

WINDOW = 32
BLOCK = 4
RHO = 0.7
GAMMA = 0.5


def make_case(rows: int, cols: int, pattern, seed: int = 0, noise: float = 0.0,
              shape: int = THREE_QUARTER):
    """Build one reconstruction case.

    Returns a dict with ``clean`` (float64 reference image), ``tile`` (uint8
    quadrant-code tile) and ``y`` (float64 sensor read-out, with pixel shape
    ``shape``, of the observed, possibly noisy, image).
    """
    clean, observed = synthetic_image(rows, cols, seed=seed, noise_sigma=noise)
    if pattern is None:
        tile = random_pattern(rows // 2, cols // 2, seed=seed)
    else:
        pr, pc = (pattern, pattern) if np.isscalar(pattern) else pattern
        tile = random_pattern(pr, pc, seed=seed)
    y = sense(observed, tile, shape)
    return dict(clean=clean, tile=tile, y=y)


BATCH_SIZES = [(256, 256), (480, 640), (768, 1024), (1080, 1920), (1536, 2048)]


def batch_cases(n_images: int = 64, seed: int = 0, sizes=None, periods=(2, 4, 8)):
    """Uneven batch: sizes drawn from ``sizes`` (rows, cols), each image with
    its own random pattern of a period drawn from ``periods``."""
    sizes = BATCH_SIZES if sizes is None else sizes
    g = np.random.default_rng(np.random.SeedSequence(seed).spawn(5)[4])
    cases = []
    for k in range(n_images):
        rows, cols = sizes[int(g.integers(0, len(sizes)))]
        period = int(periods[int(g.integers(0, len(periods)))])
        c = make_case(rows, cols, period, seed=seed * 1000 + k + 1)
        c["period"] = period
        cases.append(c)
    return cases
