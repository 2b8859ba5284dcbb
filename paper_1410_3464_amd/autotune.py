"""Tile-schedule autotuner for the step kernel.

The kernel's work item is 62 columns by `seg_rows` rows, one wavefront.  Short
items balance better on small lattices, and on a lattice that does not fill the
device they cut the time of an item's march, which is then the time of a step;
long items repeat fewer ring rows (two per item) on large ones.  The best value depends on lattice size, storage
precision and on how full the device is, so it is measured: each candidate runs
a few steps on the GPU and the fastest is kept per (size class, precision,
species count, context).  Alone, a lattice is timed by itself; for batched runs
(`fill_nodes` given) it is timed as a batch of copies holding about that many
nodes, the situation of a simulation inside a large batch, where the device is
full whatever the lattice size.  The choice changes speed only, never results.
"""
from __future__ import annotations

import math

CANDIDATES = (2, 4, 8, 12, 16, 24, 30)
_cache: dict = {}


def size_class(nx, ny):
    """Lattices whose larger side rounds to the same power of two share a choice."""
    return 1 << max(6, int(round(math.log2(max(nx, ny)))))


MAX_COPIES = 32


def tuned_seg_rows(prob, precision, stream=None, steps=20, warmup=3, fill_nodes=None):
    """seg_rows for `prob`'s size class, measured once per class on `stream`
    (a torch.cuda.Stream); later calls return the cached choice.  With
    `fill_nodes`, the candidates are timed on a batch of copies of `prob`
    (about fill_nodes nodes, at most MAX_COPIES copies) stepped by batched
    launches."""
    import torch

    from .lbrx import Batch, Lbrx

    copies = 1
    if fill_nodes:
        copies = max(1, min(MAX_COPIES, math.ceil(fill_nodes / (prob.nx * prob.ny))))
    key = (size_class(prob.nx, prob.ny), precision, prob.n_species, "batch" if fill_nodes else "alone")
    if key in _cache:
        return _cache[key]
    st = stream if stream is not None else torch.cuda.Stream()
    best, best_ms = CANDIDATES[0], float("inf")
    for h in CANDIDATES:
        sims = [Lbrx(prob, precision, stream=st.cuda_stream, seg_rows=h) for _ in range(copies)]
        run = Batch(sims) if fill_nodes else sims[0]
        run.step(warmup)
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(st)
        run.step(steps)
        b.record(st)
        st.synchronize()
        ms = a.elapsed_time(b) / steps
        if fill_nodes:
            run.close()
        for sim in sims:
            sim.close()
        if ms < best_ms:
            best, best_ms = h, ms
    _cache[key] = best
    return best


def table():
    """The choices made so far: {(size class, precision, species, context): seg_rows}."""
    return dict(_cache)
