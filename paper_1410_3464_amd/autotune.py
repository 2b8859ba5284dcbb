"""Tile-schedule autotuner for the step kernel.

The kernel's work item is 64 columns by `seg_rows` rows, one wavefront.  Short
items balance better on small lattices; long items repeat fewer ring rows (two
per item) on large ones.  The best value depends on lattice size and storage
precision, so it is measured: each candidate runs a few steps of a
representative lattice on the GPU and the fastest is kept per (size class,
precision, species count).  The choice changes speed only, never results.
"""
from __future__ import annotations

import math

CANDIDATES = (8, 12, 16, 24, 30)
_cache: dict = {}


def size_class(nx, ny):
    """Lattices whose larger side rounds to the same power of two share a choice."""
    return 1 << max(6, int(round(math.log2(max(nx, ny)))))


def tuned_seg_rows(prob, precision, stream=None, steps=20, warmup=3):
    """seg_rows for `prob`'s size class, measured once per class on `stream`
    (a torch.cuda.Stream); later calls return the cached choice."""
    import torch

    from .lbrx import Lbrx

    key = (size_class(prob.nx, prob.ny), precision, prob.n_species)
    if key in _cache:
        return _cache[key]
    st = stream if stream is not None else torch.cuda.Stream()
    best, best_ms = CANDIDATES[0], float("inf")
    for h in CANDIDATES:
        sim = Lbrx(prob, precision, stream=st.cuda_stream, seg_rows=h)
        sim.step(warmup)
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(st)
        sim.step(steps)
        b.record(st)
        st.synchronize()
        ms = a.elapsed_time(b) / steps
        sim.close()
        if ms < best_ms:
            best, best_ms = h, ms
    _cache[key] = best
    return best


def table():
    """The choices made so far: {(size class, precision, species): seg_rows}."""
    return dict(_cache)
