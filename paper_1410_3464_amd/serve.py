"""A serving loop for many independent simulations on one GPU.

Requests (a problem, a step count and a storage precision) arrive over time.
The server admits a request as soon as it has arrived and its device
footprint fits under the memory cap, keeps every admitted lattice resident,
and advances all active simulations of the same precision and species count
together: one batched launch per step (lbrx_batch_step), `tick` steps at a
time, so requests that arrive while others run join at the next tick and
their work overlaps on the device.  A request completes when its steps are
done; its fields are read back and its memory freed.

`run_plain` serves the same requests one at a time in arrival order, each
stepped alone (optionally all with the plain FP32 kernels): the reference the
batched server is compared with (latency from arrival to completion, p50 /
p99, and aggregate lattice updates per second).
"""
from __future__ import annotations

import collections
import dataclasses
import math
import time

import numpy as np

from . import workloads as W
from .autotune import tuned_seg_rows

ESZ = {"f64": 8, "f32": 4, "f16dev": 2, "bf16dev": 2}


@dataclasses.dataclass
class Request:
    rid: int
    prob: object
    steps: int
    precision: str
    arrival: float  # seconds after the start of the run
    start: float = math.nan
    finish: float = math.nan
    status: str = "pending"
    fields: dict | None = None

    @property
    def latency(self):
        return self.finish - self.arrival

    @property
    def updates(self):
        return self.prob.nx * self.prob.ny * self.steps


def poisson_requests(n, mean_interarrival, seed=0, steps=(200, 2000), sizes=(64, 1024),
                     precisions=("f32", "f16dev")):
    """n requests with exponential inter-arrival times: lattice instances of the
    many-simulations workload (sides log-uniform in `sizes`), step counts
    log-uniform in `steps`, precision drawn uniformly from `precisions`."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(mean_interarrival, size=n))
    t -= t[0]
    out = []
    for i in range(n):
        nsteps = int(round(math.exp(rng.uniform(math.log(steps[0]), math.log(steps[1])))))
        prec = precisions[int(rng.integers(len(precisions)))]
        prob = W.batch_instance(seed * 100_000 + i, smin=sizes[0], smax=sizes[1])
        out.append(Request(i, prob, nsteps, prec, float(t[i])))
    return out


def footprint_bytes(prob, precision):
    """Device memory of one simulation (both buffers of every population,
    status and code array, volumes, balance records, read-out planes)."""
    pitch = (prob.nx + 63) // 64 * 64
    plane = pitch * prob.ny
    esz = ESZ[precision]
    ns = prob.n_species
    pops = 18 * plane * esz + 10 * ((ns + 1) // 2) * plane * esz
    words = plane * 4 * (1 + (((ns + 3) // 4) if esz == 2 else 0))
    items = (pitch // 64) * ((prob.ny + 7) // 8)  # balance records: items of 8 rows or more
    return 2 * (pops + words) + plane * 8 + items * 38 * 8 + (4 + ns) * plane * 8


class Server:
    def __init__(self, hbm_cap=200e9, tick=50, autotune=True, keep_fields=False, depth=2):
        self.hbm_cap = hbm_cap
        self.tick = tick
        self.autotune = autotune
        self.keep_fields = keep_fields
        self.depth = depth  # ticks enqueued ahead of the host before it waits

    def run(self, requests):
        import torch

        from .lbrx import Batch, Lbrx, LbrxError

        stream = torch.cuda.Stream()
        if self.autotune:  # measured before the clock starts, once per size class
            for r in requests:
                tuned_seg_rows(r.prob, r.precision, stream)
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        active = {}  # rid -> (request, sim, remaining, footprint)
        batches = {}  # group -> (member rids, Batch)
        # The host runs ahead of the device by up to `depth` ticks: it waits
        # only for the oldest tick beyond that, or for the tick in which a
        # request finishes (its fields are read).  A batch replaced by a new
        # membership is closed once the ticks it was launched in are done.
        inflight = collections.deque()  # (tick, event) not yet known complete
        retired = []  # (first tick without it, Batch)
        tick_no, done_tick = 0, -1
        used = 0.0
        t0 = time.perf_counter()
        while pending or active:
            now = time.perf_counter() - t0
            while pending and pending[0].arrival <= now:
                r = pending[0]
                fp = footprint_bytes(r.prob, r.precision)
                if used + fp > self.hbm_cap and active:
                    break  # wait until memory frees up (a request larger than the cap runs alone)
                pending.popleft()
                h = tuned_seg_rows(r.prob, r.precision, stream) if self.autotune else 0
                sim = Lbrx(r.prob, r.precision, stream=stream.cuda_stream, seg_rows=h)
                r.start = time.perf_counter() - t0
                active[r.rid] = [r, sim, r.steps, fp]
                used += fp
            if not active:
                time.sleep(max(0.0, pending[0].arrival - (time.perf_counter() - t0)))
                continue
            groups = collections.defaultdict(list)
            for rid, (r, sim, rem, fp) in sorted(active.items()):
                groups[(r.precision, r.prob.n_species)].append(rid)
            for g, rids in groups.items():
                members, b = batches.get(g, ((), None))
                if tuple(rids) != members:
                    if b is not None:
                        retired.append((tick_no, b))
                    b = Batch([active[i][1] for i in rids])
                    batches[g] = (tuple(rids), b)
                k = min(self.tick, min(active[i][2] for i in rids))
                b.step(k)
                for i in rids:
                    active[i][2] -= k
            for g in [g for g in batches if g not in groups]:
                retired.append((tick_no, batches.pop(g)[1]))
            ev = torch.cuda.Event()
            ev.record(stream)
            inflight.append((tick_no, ev))
            finished = [i for i, a in active.items() if a[2] == 0]
            if finished:
                ev.synchronize()
                inflight.clear()
                done_tick = tick_no
            elif len(inflight) > self.depth:
                t_, e_ = inflight.popleft()
                e_.synchronize()
                done_tick = t_
            still = []
            for t_, b_ in retired:
                if t_ - 1 <= done_tick:
                    b_.close()
                else:
                    still.append((t_, b_))
            retired = still
            tick_no += 1
            for rid in finished:
                r, sim, _, fp = active.pop(rid)
                try:
                    sim.sync()
                    r.status = "ok"
                    if self.keep_fields:
                        r.fields = sim.fields()
                except LbrxError as e:
                    r.status = f"failed: {e}"
                r.finish = time.perf_counter() - t0
                used -= fp
                for g in list(batches):
                    if rid in batches[g][0]:
                        batches.pop(g)[1].close()
                sim.close()
        makespan = time.perf_counter() - t0
        for _, b in batches.values():
            b.close()
        for _, b in retired:
            b.close()
        return summarize(requests, makespan)


def run_plain(requests, keep_fields=False, precision=None):
    """The same requests one at a time in arrival order, each stepped alone
    (in `precision` if given, e.g. the plain FP32 kernels, else in its own)."""
    import torch

    from .lbrx import Lbrx, LbrxError

    stream = torch.cuda.Stream()
    t0 = time.perf_counter()
    for r in sorted(requests, key=lambda r: r.arrival):
        wait = r.arrival - (time.perf_counter() - t0)
        if wait > 0:
            time.sleep(wait)
        r.start = time.perf_counter() - t0
        sim = Lbrx(r.prob, precision or r.precision, stream=stream.cuda_stream)
        sim.step(r.steps)
        try:
            sim.sync()
            r.status = "ok"
            if keep_fields:
                r.fields = sim.fields()
        except LbrxError as e:
            r.status = f"failed: {e}"
        r.finish = time.perf_counter() - t0
        sim.close()
    return summarize(requests, time.perf_counter() - t0)


def summarize(requests, makespan):
    lat = np.array([r.latency for r in requests]) * 1e3
    ok = sum(r.status == "ok" for r in requests)
    upd = sum(r.updates for r in requests)
    return {"requests": len(requests), "completed": ok,
            "p50_ms": round(float(np.percentile(lat, 50)), 2), "p99_ms": round(float(np.percentile(lat, 99)), 2),
            "mlups": round(upd / makespan / 1e6, 1), "makespan_s": round(makespan, 3)}


def clone_requests(requests):
    """Fresh copies (same problems, steps, precisions and arrivals)."""
    return [Request(r.rid, r.prob, r.steps, r.precision, r.arrival) for r in requests]
