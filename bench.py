"""Throughput of the binned power-waveform path on one MI355X.

One step = one forward pass over the whole synthetic trace (gate parameters,
per-event state tracking, energies and leakage steps accumulated per time tile,
leakage prefix scan, FP32 power), with the events already resident in HBM and
the packed layout (which depends only on event times, pins and the bin width)
built before the timed region (its build time is reported under "plan").
The workload is the 1M-gate, 200M-event, 50 ps-bin configuration;
``--config`` selects another synthetic configuration.

Prints one JSON line (see the keys below). The per-kernel durations come from
HIP events recorded on the library's stream around every launch inside the
timed region.
"""
import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12          # MI355X HBM3E, bytes/s
EVENT_BYTES = 16           # per event: t int64 + slew float32 + pin/value padded to 4 bytes
EVENT_BYTES_STRICT = 13    # the same with a 1-byte pin/value
GATE_BYTES = 16            # gate parameter record read per gate
BIN_BYTES = 4              # FP32 power written per bin

WORKLOADS = {
    "C1": "1k gates, 8 cells (1-3 inputs), 100k events over 1k cycles of 1 ns, 100 ps bins",
    "C2": "1M gates, 64 cells (1-4 inputs), 200M events over 100k cycles of 1 ns, 50 ps bins, "
          "lognormal(4,2) per-gate counts, 200 clock gates",
    "C3": "5M gates, 64 cells, 1B events, Zipf(1.2) per-gate counts, 200k cycles, 100 ps bins",
    "C5": "1M gates, 64 cells, 100M events over 50k cycles, 50 ps bins (adjoint workload)",
}


# sources that decide a kernel's memory traffic: the kernels, the packed
# layout and the host's launch configuration
KERNEL_SOURCES = ("paper_2609_05960_amd/csrc/gtp_kernels.h", "paper_2609_05960_amd/csrc/gtp_device.h",
                  "paper_2609_05960_amd/csrc/gtp_scan.h",
                  "paper_2609_05960_amd/csrc/gtp_pack.h", "paper_2609_05960_amd/csrc/gtp_pack.hip",
                  "paper_2609_05960_amd/csrc/gtpower.hip")


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` on `workload` from the rocprofv3 summaries
    under profiles/ (a line 'traffic: <kernel> <workload> <bytes> src=<hash>'),
    or None when no summary matches the current kernel sources."""
    import glob
    import re
    src = kernel_source_hash()
    for f in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        with open(f) as fh:
            for line in fh:
                m = re.match(r"traffic: (\S+) (\S+) (\d+) src=([0-9a-f]+)", line.strip().strip("`"))
                if m and m.group(1) == kernel and m.group(2) == workload and m.group(4) == src:
                    return int(m.group(3))
    return None


def cpu_brand() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def bench_batched(args, gtp, torch, dev):
    """Many stimulus traces of uneven length over one netlist: the batched
    forward (one persistent launch, replayed from a HIP graph) against one
    forward per trace, same traces, same GPU."""
    import synth
    t0 = time.time()
    lib, net, traces, bin_ps = synth.make_batch(n_traces=args.batch_traces, cycles=tuple(args.batch_cycles))
    gen_s = time.time() - t0
    n_ev = sum(ev.n_events for ev in traces)
    ctx = gtp.Context(0)
    ctx.load_library(lib)
    ctx.load_netlist(torch.from_numpy(net.gate_cell).to(dev), torch.from_numpy(net.gate_out_net).to(dev),
                     torch.from_numpy(net.gate_init.view(np.int32)).to(dev), net.n_nets)
    ctx.set_params(vdd=0.8, bin_ps=bin_ps)
    tr = [tuple(torch.from_numpy(a).to(dev) for a in (ev.gate_off, ev.t, ev.pin_bit, ev.slew)) + (ev.t_end,)
          for ev in traces]
    ctx.load_traces(tr)
    load = torch.from_numpy(net.net_load).to(dev)
    lam = torch.from_numpy(net.leak_scale).to(dev)
    tot, offs = ctx.batch_bins()
    P = torch.empty(tot, dtype=torch.float32, device=dev)
    tp = time.time()
    ctx.forward_batched(load, lam, out=P, use_graph=True)  # packs every trace, records the graph
    torch.cuda.synchronize()
    plan_s = time.time() - tp
    outs = [P[int(offs[i]):int(offs[i + 1])] for i in range(len(traces))]
    stream = torch.cuda.current_stream(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn, steps):
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(steps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    def per_trace():
        for i in range(len(traces)):
            ctx.forward_trace(i, load, lam, out=outs[i])

    steps = max(2, min(args.steps, 10))
    ms_graph = timed(lambda: ctx.forward_batched(load, lam, out=P, use_graph=True), steps)
    ms_eager = timed(lambda: ctx.forward_batched(load, lam, out=P, use_graph=False), steps)
    ms_seq = timed(per_trace, steps)
    ctx.close()
    lens = [ev.t_end // 1000 for ev in traces]
    return {"workload": f"{len(traces)} traces over one {net.n_gates}-gate, {lib.n_cells}-cell netlist, "
                        f"{args.batch_cycles[0]}-{args.batch_cycles[1]} cycles of 1 ns each (drawn), "
                        f"500 events per cycle, lognormal(0,2) per-gate counts, {bin_ps} ps bins",
            "n_events": n_ev, "n_bins": int(tot), "cycles_min": int(min(lens)), "cycles_max": int(max(lens)),
            "value": n_ev / (ms_graph * 1e-3), "unit": "events/s", "ms_per_step": ms_graph,
            "eager_ms_per_step": ms_eager,
            "per_trace": {"value": n_ev / (ms_seq * 1e-3), "ms_per_step": ms_seq, "launches_per_step": 4 * len(traces)},
            "speedup_vs_per_trace": ms_seq / ms_graph, "plan_s": plan_s, "gen_s": gen_s}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="C2", choices=sorted(WORKLOADS))
    ap.add_argument("--scale", type=float, default=1.0,
                    help="shrink gates, cycles and events of the workload together (comparison runs only)")
    ap.add_argument("--algo", type=int, default=0, help="0 time-tiled, 1 one gate per thread")
    ap.add_argument("--tile-log2", type=int, default=0)
    ap.add_argument("--tile-threads", type=int, default=0, help="threads per tile workgroup (0 = library default)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target CPU work for the oracle sample")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-trace comparison")
    ap.add_argument("--batch-traces", type=int, default=64)
    ap.add_argument("--batch-cycles", type=int, nargs=2, default=[1000, 20000],
                    help="range of cycles per trace of the batched comparison")
    ap.add_argument("--autotune", default=None, help="autotune cache file (JSON lines); tune before timing")
    ap.add_argument("--calib-copy", type=int, default=0,
                    help="only run device copies of this many MiB (to scale HBM byte counters), then exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus above 1 is not supported "
                                   "(the multi-GPU sharding is a design note only)"}))
        sys.exit(2)

    import torch

    import synth
    import paper_2609_05960_amd as gtp

    dev = torch.device("cuda", 0)
    if args.calib_copy:
        n = args.calib_copy << 20
        a = torch.ones(n // 4, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calib_copy_bytes": n, "copies": 3}))
        return
    t0 = time.time()
    prob = synth.make_problem(args.config, scale=args.scale)
    gen_s = time.time() - t0
    print(f"# generated {args.config}: {prob.ev.n_events} events, {prob.net.n_gates} gates, {prob.n_bins} bins "
          f"in {gen_s:.1f} s", file=sys.stderr, flush=True)
    net, ev = prob.net, prob.ev
    ctx = gtp.Context(0)
    ctx.load_library(prob.lib)
    ctx.load_netlist(torch.from_numpy(net.gate_cell).to(dev), torch.from_numpy(net.gate_out_net).to(dev),
                     torch.from_numpy(net.gate_init.view(np.int32)).to(dev), net.n_nets)
    tens = [torch.from_numpy(a).to(dev) for a in (ev.gate_off, ev.t, ev.pin_bit, ev.slew)]
    torch.cuda.synchronize()
    tp = time.time()
    ctx.load_events(*tens, t_end=ev.t_end, validate=False)
    ctx.set_params(vdd=prob.vdd, bin_ps=prob.bin_ps, sw_mode=prob.sw_mode)
    ctx.set_tuning(algo=args.algo, bins_per_tile_log2=args.tile_log2, tile_threads=args.tile_threads)
    load = torch.from_numpy(net.net_load).to(dev)
    lam = torch.from_numpy(net.leak_scale).to(dev)
    P = torch.empty(ctx.n_bins, dtype=torch.float32, device=dev)
    if args.autotune:
        ctx.autotune(args.autotune)
    ctx.forward(load, lam, out=P)  # builds the packed layout
    torch.cuda.synchronize()
    plan_s = time.time() - tp
    plan = ctx.plan_info() if args.algo == 0 else None
    for _ in range(args.warmup):
        ctx.forward(load, lam, out=P)
    torch.cuda.synchronize()

    # ---- timed forward ---------------------------------------------------
    stream = torch.cuda.current_stream(dev)
    ctx.profile(True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        ctx.forward(load, lam, out=P)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_total = e0.elapsed_time(e1)
    kern = ctx.profile_read()
    ctx.profile(False)
    ctx.sync()
    ms_step = ms_total / args.steps
    N, G, NB = ev.n_events, net.n_gates, ctx.n_bins
    value = N * args.steps / (ms_total * 1e-3)

    kern_avg = {k: dict(launches=n, avg_ms=ms / max(n, 1), total_ms=ms) for k, (n, ms) in kern.items()}
    dom = max(kern_avg, key=lambda k: kern_avg[k]["total_ms"])
    algo_bytes = {"k_fwd_packed": EVENT_BYTES * N, "k_gate_serial": EVENT_BYTES * N + GATE_BYTES * G,
                  "k_gate_params": 24 * G, "k_gate_prep": 24 * G, "k_finalize": 28 * NB}
    dom_bytes = algo_bytes.get(dom)
    dom_ms = kern_avg[dom]["avg_ms"]
    achieved = dom_bytes / (dom_ms * 1e-3) if dom_bytes else None
    step_bytes = EVENT_BYTES * N + GATE_BYTES * G + BIN_BYTES * NB
    extra = {}
    if dom in ("k_fwd_packed", "k_gate_serial"):
        extra["strict_frac"] = EVENT_BYTES_STRICT * N / (dom_ms * 1e-3) / HBM_PEAK
    if plan is not None and dom == "k_fwd_packed":
        # bytes the packed layout actually holds per event: event word, table row
        # and slew weight,
        # unit descriptors, group offsets
        pb = 12 * plan["n_events_packed"] + 8 * 64 * plan["n_groups"] + 8 * plan["n_groups"]
        extra["packed_bytes_per_event"] = pb / max(N, 1)
        extra["packed_frac"] = pb / (dom_ms * 1e-3) / HBM_PEAK

    out = {
        "metric": "events/s into binned power waveform (fwd, fwd+adjoint); % of HBM roofline",
        "value": value,
        "unit": "events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.config}: {WORKLOADS[args.config]}"
                               + (f" (scaled by {args.scale})" if args.scale != 1.0 else ""), "n_gates": G, "n_events": N,
                   "n_bins": NB, "bin_ps": prob.bin_ps, "t_end_ps": ev.t_end, "algo": args.algo,
                   "tuning": ctx.get_tuning()},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": (achieved / 1e9) if achieved else None,
                     "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                     "frac": (achieved / HBM_PEAK) if achieved else None,
                     "traffic": measured_traffic(dom, args.config),
                     "algorithmic_bytes_per_launch": dom_bytes, "algorithmic_bytes_per_event": EVENT_BYTES,
                     "avg_launch_ms": dom_ms, **extra},
        "step_hbm_frac": step_bytes / (ms_step * 1e-3) / HBM_PEAK,
        "kernels": kern_avg,
        "kernel_src": kernel_source_hash(),
        "plan_s": plan_s,
        "plan": plan,
        "gen_s": gen_s,
    }

    # ---- events -> waveform: plan, packed layout and forward together -------
    # (the layout is rebuilt every step: gtp_load_events drops it, the forward
    # rebuilds it; the builder waits on the host, so the step is timed with
    # the host clock around device-synchronised steps)
    if args.algo == 0:
        e2w_steps = max(2, min(args.steps, 5))
        times = []
        for it in range(e2w_steps + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.load_events(*tens, t_end=ev.t_end, validate=False)
            ctx.forward(load, lam, out=P)
            torch.cuda.synchronize()
            if it > 0:   # the first step also grows the builder's workspace
                times.append(time.perf_counter() - t0)
        ms_e2w = 1e3 * sum(times) / len(times)
        pk = ctx.plan_info()
        out_e2w = {"value": N / (ms_e2w * 1e-3), "unit": "events/s", "ms_per_step": ms_e2w, "steps": e2w_steps,
                   "pack_ms": pk["pack_ms"],
                   "frac": EVENT_BYTES * N / (ms_e2w * 1e-3) / HBM_PEAK,
                   "note": "events in the caller's gate-major layout to FP32 waveform: lane-block plan, packed "
                           "layout (partition, carried-in state, per-event state, table rows, slew weights) and "
                           "the forward, every step"}
    # ---- forward + adjoint -------------------------------------------------
    if not args.no_adjoint:
        beta = float(1.0 / (0.05 * P.double().mean().item()))
        gP = torch.empty_like(P)
        for _ in range(2):
            ctx.forward(load, lam, out=P)
            z = beta * P  # gradient of the smooth peak-power loss: softmax(beta P)
            torch.exp(z - z.max(), out=gP)
            gP.div_(gP.sum())
            ctx.adjoint(load, lam, gP)
        torch.cuda.synchronize()
        ctx.profile(True)
        e0.record(stream)
        for _ in range(args.steps):
            ctx.forward(load, lam, out=P)
            z = beta * P  # gradient of the smooth peak-power loss: softmax(beta P)
            torch.exp(z - z.max(), out=gP)
            gP.div_(gP.sum())
            ctx.adjoint(load, lam, gP)
        e1.record(stream)
        torch.cuda.synchronize()
        kern_fa = ctx.profile_read()
        ctx.profile(False)
        ms_fa = e0.elapsed_time(e1) / args.steps
        out["fwd_adjoint"] = {"value": N / (ms_fa * 1e-3), "unit": "events/s", "ms_per_step": ms_fa,
                              "kernels": {k: dict(launches=n, avg_ms=ms / max(n, 1)) for k, (n, ms) in kern_fa.items()}}

    if args.algo == 0:
        out["events_to_waveform"] = out_e2w
    # ---- batched traces: one persistent graph launch vs per-trace launches --
    if not args.no_batched:
        out["batched"] = bench_batched(args, gtp, torch, dev)

    # ---- CPU oracle on a bounded sample ------------------------------------
    if not args.no_cpu:
        import oracle
        O = oracle.get()
        counts = np.diff(ev.gate_off)
        cum = np.cumsum(counts)
        # calibrate on ~10% of the events, then size the sample for about --cpu-seconds
        m = int(np.searchsorted(cum, max(1, N // 10))) + 1
        m = min(m, G)
        t1 = time.time()
        O.forward(prob, gates=np.arange(m), nthreads=0)
        rate = cum[m - 1] / max(time.time() - t1, 1e-6)
        target = min(N, int(rate * args.cpu_seconds))
        m = int(np.searchsorted(cum, target)) + 1
        m = min(m, G)
        t1 = time.time()
        O.forward(prob, gates=np.arange(m), nthreads=0)
        dt = time.time() - t1
        ns = int(cum[m - 1])
        out["cpu_baseline"] = {"value": ns / dt, "unit": "events/s", "cores": O.max_threads(), "kind": "oracle",
                               "sample": f"gates 0..{m - 1} of {args.config} ({ns} events, all {NB} bins), "
                                         f"FP64, {dt:.1f} s", "cpu": cpu_brand()}
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
