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
import sys
import time

import numpy as np

from . import workloads as W
from .autotune import tuned_seg_rows

ESZ = {"f64": 8, "f32": 4, "f16dev": 2, "bf16dev": 2}


@dataclasses.dataclass
class Request:
    rid: int
    prob: object  # the problem, or None: generated from `spec` when admitted
    steps: int
    precision: str
    arrival: float  # seconds after the start of the run
    start: float = math.nan
    finish: float = math.nan
    status: str = "pending"
    fields: dict | None = None
    spec: tuple | None = None  # (seed, smin, smax) of a batch_instance made on admission
    side: int = 0

    @property
    def latency(self):
        return self.finish - self.arrival

    @property
    def dims(self):
        """(nx, ny, species) without generating the problem."""
        if self.prob is not None:
            return self.prob.nx, self.prob.ny, self.prob.n_species
        return self.side, self.side, 4

    @property
    def updates(self):
        nx, ny, _ = self.dims
        return nx * ny * self.steps

    def problem(self):
        """The problem (generated now for a request that carries only its spec;
        not kept, so that a long stream of requests holds no host arrays)."""
        return self.prob if self.prob is not None else W.batch_instance(*self.spec)


def poisson_requests(n, mean_interarrival, seed=0, steps=(200, 2000), sizes=(64, 1024),
                     precisions=("f32", "f16dev"), lazy=False):
    """n requests with exponential inter-arrival times: lattice instances of the
    many-simulations workload (sides log-uniform in `sizes`), step counts
    log-uniform in `steps`, precision drawn uniformly from `precisions`.  With
    `lazy`, a request carries only the seed of its instance, generated when it
    is admitted."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(mean_interarrival, size=n))
    t -= t[0]
    out = []
    for i in range(n):
        nsteps = int(round(math.exp(rng.uniform(math.log(steps[0]), math.log(steps[1])))))
        prec = precisions[int(rng.integers(len(precisions)))]
        spec = (seed * 100_000 + i, sizes[0], sizes[1])
        if lazy:
            out.append(Request(i, None, nsteps, prec, float(t[i]), spec=spec, side=W.batch_instance_side(*spec)))
        else:
            out.append(Request(i, W.batch_instance(*spec), nsteps, prec, float(t[i])))
    return out


def footprint_bytes(prob, precision):
    """Device memory of one simulation (both buffers of every population,
    status and code array, volumes, balance records, read-out planes); `prob`
    is a problem or a Request."""
    nx, ny, ns = prob.dims if isinstance(prob, Request) else (prob.nx, prob.ny, prob.n_species)
    pitch = (nx + 63) // 64 * 64
    plane = pitch * ny
    esz = ESZ[precision]
    pops = 18 * plane * esz + 10 * ((ns + 1) // 2) * plane * esz
    words = plane * 4 * (1 + (((ns + 3) // 4) if esz == 2 else 0))
    items = -(-nx // 62) * ((ny + 1) // 2)  # balance records: items of 62 columns, 2 rows or more
    return 2 * (pops + words) + plane * 8 + items * 38 * 8 + (4 + ns) * plane * 8


def _progress(tag, t0, last, every, requests, active=0):
    """A progress line on stderr at most every `every` seconds of the run."""
    now = time.perf_counter() - t0
    if every and now - last >= every:
        done = sum(1 for r in requests if r.status != "pending")
        print(f"# {tag}: t={now:.0f}s completed={done}/{len(requests)} active={active}", file=sys.stderr, flush=True)
        return now
    return last


class Server:
    def __init__(self, hbm_cap=200e9, tick=50, autotune=True, keep_fields=False, depth=2, progress=0.0):
        self.hbm_cap = hbm_cap
        self.tick = tick
        self.autotune = autotune
        self.keep_fields = keep_fields
        self.depth = depth  # ticks enqueued ahead of the host before it waits
        self.progress = progress  # seconds between progress lines (0: none)

    def run(self, requests):
        import torch

        from .lbrx import Batch, Lbrx, LbrxError

        stream = torch.cuda.Stream()
        if self.autotune:  # measured before the clock starts, once per size class
            seen = set()
            for r in requests:
                nx, ny, ns = r.dims
                key = (max(nx, ny), r.precision, ns) if r.prob is None else id(r)
                if key not in seen:
                    seen.add(key)
                    tuned_seg_rows(r.problem(), r.precision, stream)
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
        last = 0.0
        while pending or active:
            last = _progress("serve", t0, last, self.progress, requests, len(active))
            now = time.perf_counter() - t0
            while pending and pending[0].arrival <= now:
                r = pending[0]
                fp = footprint_bytes(r, r.precision)
                if used + fp > self.hbm_cap and active:
                    break  # wait until memory frees up (a request larger than the cap runs alone)
                pending.popleft()
                prob = r.problem()
                h = tuned_seg_rows(prob, r.precision, stream) if self.autotune else 0
                sim = Lbrx(prob, r.precision, stream=stream.cuda_stream, seg_rows=h)
                del prob
                r.start = time.perf_counter() - t0
                active[r.rid] = [r, sim, r.steps, fp]
                used += fp
            if not active:
                time.sleep(max(0.0, pending[0].arrival - (time.perf_counter() - t0)))
                continue
            groups = collections.defaultdict(list)
            for rid, (r, sim, rem, fp) in sorted(active.items()):
                groups[(r.precision, r.dims[2])].append(rid)
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


def run_plain(requests, keep_fields=False, precision=None, progress=0.0):
    """The same requests one at a time in arrival order, each stepped alone
    (in `precision` if given, e.g. the plain FP32 kernels, else in its own)."""
    import torch

    from .lbrx import Lbrx, LbrxError

    stream = torch.cuda.Stream()
    t0 = time.perf_counter()
    last = 0.0
    for r in sorted(requests, key=lambda r: r.arrival):
        last = _progress("plain", t0, last, progress, requests)
        wait = r.arrival - (time.perf_counter() - t0)
        if wait > 0:
            time.sleep(wait)
        r.start = time.perf_counter() - t0
        sim = Lbrx(r.problem(), precision or r.precision, stream=stream.cuda_stream)
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
    failed = collections.Counter(r.precision for r in requests if r.status.startswith("failed"))
    return {"requests": len(requests), "completed": ok, "failed_by_precision": dict(failed),
            "p50_ms": round(float(np.percentile(lat, 50)), 2), "p99_ms": round(float(np.percentile(lat, 99)), 2),
            "mlups": round(upd / makespan / 1e6, 1), "makespan_s": round(makespan, 3)}


def clone_requests(requests):
    """Fresh copies (same problems, steps, precisions and arrivals)."""
    return [Request(r.rid, r.prob, r.steps, r.precision, r.arrival, spec=r.spec, side=r.side) for r in requests]
