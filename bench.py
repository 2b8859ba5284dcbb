"""Throughput of the coupled reactive-transport LB step on one MI355X.

Workload: the porous-medium generator at 4096 x 4096 (porosity 0.55, 20% of the
solid dissolvable, 30% of the pore space vapour, two flow components, four
species, two homogeneous and two surface reactions), FP32 by default.  One step
is one launch of the fused step kernel over the whole lattice; the populations
are resident in HBM before the timed region starts.

Prints one JSON line: MLUPS (nx*ny*steps/s/1e6), the HBM roofline of the step
kernel (algorithmic bytes per launch / kernel time from HIP events on the
library's stream), the FP64 CPU oracle timed on a bounded sample of the same
lattice on the host cores, and two many-simulation comparisons: 256 porous
instances stepped together by batched launches against one at a time
("batched"), and Poisson-arriving requests served by the continuous-batching
loop against plain one-at-a-time runs ("serving").
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
FILL_NODES = 4_000_000  # batched item heights are tuned on copies holding about this many nodes
METRIC = "coupled-step MLUPS & %HBM roofline on 1 MI355X; serving p50/p99 vs plain"


def algorithmic_bytes(F, prob, esz):
    """Bytes one step must move at minimum: every flow population of a fluid node
    read and written once, every solute population of a liquid node read and
    written once, the node-type byte read and written, and the FP64 solid /
    precipitate volume read and written at liquid-solid interface nodes (with
    16-bit storage also the solute reference codes of liquid nodes)."""
    t = F["type"]
    fluid = t == 0
    liq = F["liquid"].astype(bool)
    ns = prob.n_species
    reactive = (t == 2) | (t == 3)
    # D2Q5 neighbours (periodicity as in the problem)
    def shifted(m, dx, dy):
        out = np.roll(m, (dy, dx), axis=(0, 1))
        if not prob.periodic_x:
            if dx > 0: out[:, :dx] = False
            if dx < 0: out[:, dx:] = False
        if not prob.periodic_y:
            if dy > 0: out[:dy, :] = False
            if dy < 0: out[dy:, :] = False
        return out
    near_liq = np.zeros_like(liq)
    near_rs = np.zeros_like(liq)
    for dx, dy in ((1, 0), (-1, 0), (0, 1), (0, -1)):
        near_liq |= shifted(liq, dx, dy)
        near_rs |= shifted(reactive, dx, dy)
    interface = (reactive & near_liq) | (liq & near_rs)
    n = t.size
    b = (int(fluid.sum()) * 36 * esz + int(liq.sum()) * 10 * ns * esz + 2 * n + 16 * int(interface.sum()))
    if esz == 2 and ns > 0:
        # 16-bit storage: the solute reference codes, one 32-bit word per four species, read and written
        b += int(liq.sum()) * 8 * ((ns + 3) // 4)
    counts = dict(fluid=int(fluid.sum()), liquid=int(liq.sum()), interface=int(interface.sum()), nodes=n)
    return b, counts


def measured_traffic(precision, n):
    """HBM bytes per step-kernel launch from the committed rocprofv3 counter
    summary (calibrated FETCH_SIZE + WRITE_SIZE), or None when there is none for
    this precision and size or the kernel source has changed since."""
    import hashlib

    path = os.path.join(ROOT, "profiles", f"k_step_{precision}_porous{n}_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    src = open(os.path.join(ROOT, rec["kernel_source"]), "rb").read()
    if hashlib.sha256(src).hexdigest() != rec["kernel_source_sha256"]:
        return None
    return rec["traffic_bytes_per_launch"]


def serving(n, interarrival, steps=(200, 2000), cap_gb=200.0, mode="both", progress=30.0):
    """Poisson arrivals of many-simulation requests (square porous lattices of
    side 64-1024, step counts log-uniform in `steps`, FP32 or FP16-deviation
    storage drawn per request), served by the batched loop (admission capped at
    `cap_gb` of device memory) and, for comparison, the same requests one at a
    time with plain FP32 runs.  `mode` runs both sides, or only one ("batched",
    "plain"): the same seed gives the same requests, so a long stream can be
    measured in two runs."""
    from paper_1410_3464_amd import serve

    reqs = serve.poisson_requests(n, interarrival, seed=11, steps=steps, lazy=True)
    out = {"workload": f"{n} requests, Poisson arrivals every {interarrival * 1e3:.0f} ms on average "
                       f"(over {reqs[-1].arrival:.0f} s), porous lattices 64^2-1024^2, {steps[0]}-{steps[1]} steps, "
                       f"f32 or f16dev, admission cap {cap_gb:g} GB; plain: one at a time in f32"}
    if mode in ("both", "batched"):
        out["batched"] = serve.Server(tick=60, hbm_cap=cap_gb * 1e9, progress=progress).run(reqs)
        print(f"# serving batched {out['batched']}", file=sys.stderr, flush=True)
    if mode in ("both", "plain"):
        out["plain"] = serve.run_plain(serve.clone_requests(reqs), precision="f32", progress=progress)
        print(f"# serving plain {out['plain']}", file=sys.stderr, flush=True)
    span = reqs[-1].arrival
    if span < 540 or steps != (1000, 50000) or cap_gb != 200.0:
        out["note"] = ("a short stand-in for the 10-minute stream of 1000-50000-step requests under a 200 GB cap "
                       "(bench.py --serve-requests 600 --serve-interarrival-ms 1000 --serve-steps 1000,50000 runs it)")
    if mode == "both":
        out["p50_speedup"] = round(out["plain"]["p50_ms"] / out["batched"]["p50_ms"], 2)
        out["p99_speedup"] = round(out["plain"]["p99_ms"] / out["batched"]["p99_ms"], 2)
        out["mlups_ratio"] = round(out["batched"]["mlups"] / out["plain"]["mlups"], 2)
    return out


def batched(n_inst, steps, warmup=30, plain_warmup=30):
    """Many independent simulations: n_inst FP32 instances of the porous-medium
    generator (square sides log-uniform in 64-1024, porosity uniform in
    0.4-0.8, rate constants log-uniform in 1e-6-1e-1), advanced together by one
    launch per step (HIP graphs of 30 steps; item heights from the autotuner,
    timed on batches of copies that fill the device), against the same instances run one after the other, each alone with the
    default item height.  Both sides time `steps` steps per instance after
    warm-up steps; creating the simulations is outside the timed regions."""
    import torch

    from paper_1410_3464_amd import workloads as W
    from paper_1410_3464_amd.autotune import table, tuned_seg_rows
    from paper_1410_3464_amd.lbrx import Batch, Lbrx, LbrxError

    probs = [W.batch_instance(50_000 + i) for i in range(n_inst)]
    nodes = sum(p.nx * p.ny for p in probs)
    st = torch.cuda.Stream()
    seg = [tuned_seg_rows(p, "f32", st, fill_nodes=FILL_NODES) for p in probs]
    sims = [Lbrx(p, "f32", stream=st.cuda_stream, seg_rows=h) for p, h in zip(probs, seg)]
    b = Batch(sims)
    b.step(warmup)
    st.synchronize()
    t0 = time.perf_counter()
    b.step(steps)
    st.synchronize()
    wall_b = time.perf_counter() - t0
    b.close()
    # an instance can become numerically unstable (its fields are then
    # meaningless); both sides run it all the same and the count is reported
    failed_b = []
    for i, s in enumerate(sims):
        try:
            s.sync()
        except LbrxError as e:
            failed_b.append((probs[i].name, str(e)))
        s.close()
    del sims
    print(f"# batched: {n_inst} instances, {nodes} nodes, {wall_b / steps * 1e3:.3f} ms per step",
          file=sys.stderr, flush=True)
    wall_p = 0.0
    failed_p = []
    t_last = time.perf_counter()
    for i, p in enumerate(probs):
        if time.perf_counter() - t_last > 30:
            t_last = time.perf_counter()
            print(f"# one at a time: {i}/{n_inst} instances done", file=sys.stderr, flush=True)
        s = Lbrx(p, "f32", stream=st.cuda_stream)
        s.step(plain_warmup)
        st.synchronize()
        t0 = time.perf_counter()
        s.step(steps)
        st.synchronize()
        wall_p += time.perf_counter() - t0
        try:
            s.sync()
        except LbrxError:
            failed_p.append(p.name)
        s.close()
    mb = nodes * steps / wall_b / 1e6
    mp = nodes * steps / wall_p / 1e6
    print(f"# batched {mb:.1f} MLUPS, one at a time {mp:.1f} MLUPS", file=sys.stderr, flush=True)
    return {
        "workload": f"{n_inst} FP32 porous instances, sides log-uniform 64-1024 "
                    f"({nodes} nodes in all), {steps} timed steps each",
        "batched_mlups": round(mb, 1), "one_at_a_time_mlups": round(mp, 1),
        "ratio": round(mb / mp, 2),
        "batched_ms_per_step": round(wall_b / steps * 1e3, 3),
        "one_at_a_time_s": round(wall_p, 3),
        "seg_rows_by_size_class": {f"{k[0]}": v for k, v in table().items() if k[1] == "f32" and k[3] == "batch"},
        "unstable_instances": {"batched": [f"{n}: {e}" for n, e in failed_b], "one_at_a_time": failed_p},
        **({} if (n_inst, steps) == (256, 5000) else
           {"note": "a shorter stand-in for 256 instances x 5000 steps (bench.py --batch-instances 256 "
                    "--batch-steps 5000 runs it)"}),
    }


def precision_comparison(prob, precision, main_mlups, steps, warmup):
    """The same lattice stepped with another storage precision (16-bit
    deviations by default): its rate, the ratio to the main precision's and
    its algorithmic roofline fraction."""
    import torch

    from paper_1410_3464_amd.lbrx import Lbrx

    esz = {"f64": 8, "f32": 4, "f16dev": 2, "bf16dev": 2}[precision]
    st = torch.cuda.Stream()
    sim = Lbrx(prob, precision, stream=st.cuda_stream)
    sim.step(warmup)
    sim.sync()
    b_alg, _ = algorithmic_bytes(sim.fields(), prob, esz)
    a = torch.cuda.Event(enable_timing=True)
    e = torch.cuda.Event(enable_timing=True)
    st.synchronize()
    t0 = time.perf_counter()
    a.record(st)
    sim.step(steps)
    e.record(st)
    st.synchronize()
    wall = time.perf_counter() - t0
    sim.sync()
    kern_ms = a.elapsed_time(e) / steps
    sim.close()
    mlups = prob.nx * prob.ny * steps / wall / 1e6
    print(f"# {precision}: {mlups:.1f} MLUPS", file=sys.stderr, flush=True)
    return {"dtype": precision, "value": round(mlups, 1), "unit": "MLUPS",
            "ms_per_step": round(wall / steps * 1e3, 4), "ratio_to_main": round(mlups / main_mlups, 3),
            "roofline_frac": round(b_alg / (kern_ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
            "traffic": None if measured_traffic(precision, prob.nx) is None
            else round(measured_traffic(precision, prob.nx) / 1e9, 4)}


def cpu_info():
    """The host's CPU model, logical CPU count and the CPUs this process may use."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    return model, os.cpu_count() or 1, avail


def cpu_baseline(prob, steps, threads=1):
    """The FP64 oracle, as it stands, on the host: `steps` steps of `prob` after
    one untimed step, on `threads` threads (its node loops run in parallel, its
    balances serially in node order: the result is the single-thread one)."""
    from oracle import OracleSim, build_oracle

    build_oracle()
    s = OracleSim(prob, threads=threads)
    s.step(1)  # first touch of the arrays
    t0 = time.perf_counter()
    s.step(steps)
    dt = time.perf_counter() - t0
    s.close()
    return prob.nx * prob.ny * steps / dt / 1e6, dt


def cpu_threads():
    """Threads for the all-core oracle run: OMP_NUM_THREADS if set, else the
    CPUs this process may use."""
    _, _, avail = cpu_info()
    env = os.environ.get("OMP_NUM_THREADS", "")
    return max(1, min(int(env), avail) if env.isdigit() and int(env) > 0 else avail)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--precision", default="f32", choices=["f32", "f64", "f16dev", "bf16dev"])
    ap.add_argument("--size", type=int, default=4096)
    ap.add_argument("--cpu-steps", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-full", action="store_true",
                    help="also time the oracle on the 1024x512 porous medium (200 steps) and the 4096^2 one "
                         "(10 steps), single-threaded and on all cores")
    ap.add_argument("--serve-requests", type=int, default=48,
                    help="requests of the serving comparison (0: skip it)")
    ap.add_argument("--serve-interarrival-ms", type=float, default=15.0)
    ap.add_argument("--serve-steps", default="200,2000", help="step-count range of the requests")
    ap.add_argument("--serve-cap-gb", type=float, default=200.0)
    ap.add_argument("--serve-mode", default="both", choices=["both", "batched", "plain"])

    ap.add_argument("--batch-instances", type=int, default=256,
                    help="instances of the many-simulations comparison (0: skip it)")
    ap.add_argument("--batch-steps", type=int, default=200)
    ap.add_argument("--compare-precision", default="f16dev",
                    help="storage precision timed on the same lattice beside the main one ('' skips it)")
    ap.add_argument("--copy-probe-gb", type=float, default=0.0,
                    help="run a plain device-to-device copy of this many GB first (counter calibration)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "lbrx steps each simulation on one GPU and has no multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1410_3464_amd import workloads as W
    from paper_1410_3464_amd.lbrx import Lbrx

    assert torch.cuda.is_available(), "no GPU visible"
    torch.cuda.set_device(0)
    if args.copy_probe_gb > 0:
        n_el = int(args.copy_probe_gb * 1e9) // 4
        src = torch.ones(n_el, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"# copy probe: {n_el * 4} bytes read and written", file=sys.stderr, flush=True)
        del src, dst
    t_gen = time.perf_counter()
    prob = W.config2(n=args.size)
    print(f"# generated {prob.name} in {time.perf_counter() - t_gen:.1f}s", file=sys.stderr, flush=True)
    # a dedicated (default-priority) stream: the library enqueues on it and the
    # timing events are recorded on it
    stream = torch.cuda.Stream()
    sim = Lbrx(prob, args.precision, stream=stream.cuda_stream)
    esz = {"f64": 8, "f32": 4, "f16dev": 2, "bf16dev": 2}[args.precision]

    sim.step(args.warmup)
    sim.sync()
    F = sim.fields()
    bytes_per_step, counts = algorithmic_bytes(F, prob, esz)
    print(f"# warmup done: {counts}", file=sys.stderr, flush=True)

    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    stream.synchronize()
    t0 = time.perf_counter()
    start.record(stream)
    sim.step(args.steps)
    end.record(stream)
    stream.synchronize()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sim.sync()  # raises on a numerical failure during the timed steps
    wall = t1 - t0
    kern_ms = start.elapsed_time(end) / args.steps
    F2 = sim.fields()
    b2, counts2 = algorithmic_bytes(F2, prob, esz)
    b_alg = 0.5 * (bytes_per_step + b2)

    n = prob.nx * prob.ny
    mlups = n * args.steps / wall / 1e6
    achieved = b_alg / (kern_ms * 1e-3) / 1e9
    traffic = measured_traffic(args.precision, args.size)
    out = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic",
        "config": {
            "workload": f"{prob.name} porous medium (porosity 0.55, 30% of pores vapour, 2 flow components, "
                        f"{prob.n_species} species, 2 homogeneous + 2 surface reactions)",
            "nx": prob.nx, "ny": prob.ny, "species": prob.n_species,
            "fluid_frac": round(counts["fluid"] / n, 4), "liquid_frac": round(counts["liquid"] / n, 4),
            "interface_frac": round(counts["interface"] / n, 4),
            "bytes_per_node": round(b_alg / n, 2),
            "mflups": round(mlups * 0.5 * (counts["fluid"] + counts2["fluid"]) / n, 1),
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 4),
            "traffic": None if traffic is None else round(traffic / 1e9, 4),
            "traffic_unit": "GB per launch (rocprofv3 FETCH_SIZE x 2 + WRITE_SIZE x 1, copy-calibrated)",
            "traffic_gbs": None if traffic is None else round(traffic / (kern_ms * 1e-3) / 1e9, 1),
            "traffic_frac": None if traffic is None else round(traffic / (kern_ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
            "waste": None if traffic is None else round(traffic / b_alg, 3),
            "kernel_ms": round(kern_ms, 4),
            "alg_bytes_per_launch": int(b_alg),
        },
        "cpu_baseline": None,
    }
    sim.close()
    del sim
    if args.compare_precision and args.compare_precision != args.precision:
        out["precision"] = precision_comparison(prob, args.compare_precision, mlups, args.steps, args.warmup)
    if args.batch_instances > 0:
        out["batched"] = batched(args.batch_instances, args.batch_steps)
    if args.serve_requests > 0:
        lo, hi = (int(v) for v in args.serve_steps.split(","))
        out["serving"] = serving(args.serve_requests, args.serve_interarrival_ms / 1e3, steps=(lo, hi),
                                 cap_gb=args.serve_cap_gb, mode=args.serve_mode)
    if not args.no_cpu:
        model, nproc, avail = cpu_info()
        nt = cpu_threads()
        m1, dt1 = cpu_baseline(prob, args.cpu_steps, 1)
        mt, dtt = cpu_baseline(prob, args.cpu_steps, nt)
        out["cpu_baseline"] = {
            "value": round(mt, 3), "unit": "MLUPS", "cores": nt, "kind": "oracle",
            "sample": f"{args.cpu_steps} FP64 oracle steps of the same {prob.nx}x{prob.ny} lattice after one "
                      f"untimed step, node loops on {nt} threads ({dtt:.1f}s)",
            "single_thread": {"value": round(m1, 3), "unit": "MLUPS", "cores": 1, "seconds": round(dt1, 2)},
            "cpu_model": model, "nproc": nproc, "cpus_available": avail,
        }
        if args.cpu_full:
            from paper_1410_3464_amd import workloads as W
            full = {}
            for tag, p, n in (("porous-1024x512", W.config1(), 200), (prob.name, prob, 10)):
                a1, s1 = cpu_baseline(p, n, 1)
                an, sn = cpu_baseline(p, n, nt)
                full[tag] = {"steps": n, "single_thread_mlups": round(a1, 3), "single_thread_s": round(s1, 2),
                             "threads": nt, "threaded_mlups": round(an, 3), "threaded_s": round(sn, 2)}
                print(f"# cpu {tag}: {full[tag]}", file=sys.stderr, flush=True)
            out["cpu_baseline"]["full"] = full
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
