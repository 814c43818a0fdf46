"""Parallel runs of the FP64 CPU oracle over chosen windows (test helper).

The oracle is test infrastructure; this module only spreads its per-window
work over host processes (windows are independent) and gathers the blocks
and selection sequences.
"""
from __future__ import annotations

import multiprocessing as mp
import os

import numpy as np

from oracle import ljsde_oracle as O


def _work(args):
    y, tile, blocks, kw = args
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except Exception:  # pragma: no cover
        pass
    out, tr = O.reconstruct(y, tile, blocks=blocks, traces=True, **kw)
    B = kw.get("B", 4)
    return [(bi, bj, out[B * bi:B * bi + B, B * bj:B * bj + B], np.array(tr[(bi, bj)].picks, np.int16),
             np.array(tr[(bi, bj)].gap)) for bi, bj in blocks]


def run_blocks(y, tile, blocks, procs=None, **kw):
    """Oracle (RL-JSDE form unless ``form`` is given) on ``blocks``; returns
    {(bi, bj): (block, picks, top-2 gaps)}."""
    kw.setdefault("form", "RL")
    procs = procs or min(os.cpu_count() or 1, 16)
    blocks = list(blocks)
    chunks = [blocks[k::procs] for k in range(procs)]
    with mp.get_context("fork").Pool(procs) as pool:
        parts = pool.map(_work, [(y, tile, ch, kw) for ch in chunks if ch])
    return {(bi, bj): (blk, pk, gp) for part in parts for bi, bj, blk, pk, gp in part}


_SHARED = []  # inputs of run_many, inherited by the forked workers


def _work_many(args):
    k, blocks, kw = args
    y, tile = _SHARED[k]
    return k, _work((y, tile, blocks, kw))


def run_many(jobs, procs=None, chunk=32, **kw):
    """Oracle on several images at once: ``jobs`` is a list of (y, tile,
    blocks); returns one {(bi, bj): (block, picks, top-2 gaps)} per job. The
    images reach the workers by fork, not by pickling."""
    kw.setdefault("form", "RL")
    procs = procs or min(os.cpu_count() or 1, 16)
    _SHARED[:] = [(y, tile) for y, tile, _ in jobs]
    tasks = []
    for k, (_, _, blocks) in enumerate(jobs):
        blocks = list(blocks)
        tasks += [(k, blocks[i:i + chunk], kw) for i in range(0, len(blocks), chunk)]
    try:
        with mp.get_context("fork").Pool(procs) as pool:
            parts = pool.map(_work_many, tasks, chunksize=1)
    finally:
        _SHARED[:] = []
    out = [dict() for _ in jobs]
    for k, part in parts:
        for bi, bj, blk, pk, gp in part:
            out[k][(bi, bj)] = (blk, pk, gp)
    return out


def centre_blocks(n_blocks_r: int, n_blocks_c: int, crop_px: int, B: int = 4):
    nr, nc = crop_px // B, crop_px // B
    r0, c0 = (n_blocks_r - nr) // 2, (n_blocks_c - nc) // 2
    return [(bi, bj) for bi in range(r0, r0 + nr) for bj in range(c0, c0 + nc)]


def sample_blocks(n_blocks_r: int, n_blocks_c: int, n: int, seed: int = 0):
    """Random blocks plus the four corner blocks and one edge block per side."""
    rng = np.random.default_rng(seed)
    flat = rng.choice(n_blocks_r * n_blocks_c, size=min(n, n_blocks_r * n_blocks_c), replace=False)
    s = {divmod(int(f), n_blocks_c) for f in flat}
    s |= {(0, 0), (0, n_blocks_c - 1), (n_blocks_r - 1, 0), (n_blocks_r - 1, n_blocks_c - 1),
          (0, n_blocks_c // 2), (n_blocks_r - 1, n_blocks_c // 3), (n_blocks_r // 2, 0), (n_blocks_r // 3, n_blocks_c - 1)}
    return sorted(s)
