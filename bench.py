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
# device bytes per event of a batched trace group: the caller's events
# (13 B), the packed layout (about 16 B) and a share of the layout builder's
# temporaries
BATCH_BYTES_PER_EVENT = 36

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


def log(msg):
    print(f"# {msg}", file=sys.stderr, flush=True)


def open_problem(gtp, torch, dev, prob, algo=0, tile_log2=0, tile_threads=0):
    """A context with prob's library, netlist, events (on the device) and
    parameters; returns (ctx, device event tensors, load, leak scale)."""
    net, ev = prob.net, prob.ev
    ctx = gtp.Context(0)
    ctx.load_library(prob.lib)
    ctx.load_netlist(torch.from_numpy(net.gate_cell).to(dev), torch.from_numpy(net.gate_out_net).to(dev),
                     torch.from_numpy(net.gate_init.view(np.int32)).to(dev), net.n_nets)
    tens = [torch.from_numpy(a).to(dev) for a in (ev.gate_off, ev.t, ev.pin_bit, ev.slew)]
    ctx.load_events(*tens, t_end=ev.t_end, validate=False)
    ctx.set_params(vdd=prob.vdd, bin_ps=prob.bin_ps, sw_mode=prob.sw_mode)
    ctx.set_tuning(algo=algo, bins_per_tile_log2=tile_log2, tile_threads=tile_threads)
    load = torch.from_numpy(net.net_load).to(dev)
    lam = torch.from_numpy(net.leak_scale).to(dev)
    return ctx, tens, load, lam


def timed_forward(ctx, torch, stream, load, lam, P, steps):
    """ms per forward (HIP events on the stream) and the per-kernel averages."""
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ctx.profile(True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(steps):
        ctx.forward(load, lam, out=P)
    e1.record(stream)
    torch.cuda.synchronize()
    kern = ctx.profile_read()
    ctx.profile(False)
    ctx.sync()
    kern_avg = {k: dict(launches=n, avg_ms=ms / max(n, 1), total_ms=ms) for k, (n, ms) in kern.items()}
    return e0.elapsed_time(e1) / steps, kern_avg


def timed_fwd_adjoint(ctx, torch, stream, load, lam, P, steps):
    """ms per forward + smooth-peak loss gradient + adjoint step."""
    beta = float(1.0 / (0.05 * P.double().mean().item()))
    gP = torch.empty_like(P)

    def step():
        ctx.forward(load, lam, out=P)
        z = beta * P  # gradient of the smooth peak-power loss: softmax(beta P)
        torch.exp(z - z.max(), out=gP)
        gP.div_(gP.sum())
        ctx.adjoint(load, lam, gP)

    for _ in range(2):
        step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ctx.profile(True)
    e0.record(stream)
    for _ in range(steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    kern = ctx.profile_read()
    ctx.profile(False)
    return e0.elapsed_time(e1) / steps, {k: dict(launches=n, avg_ms=ms / max(n, 1)) for k, (n, ms) in kern.items()}


def events_to_waveform(ctx, torch, tens, t_end, load, lam, P, steps):
    """Plan, packed layout and forward together, every step (the builder
    waits on the host, so steps are timed with the host clock around
    device-synchronised steps; the first step also grows the workspaces)."""
    times = []
    for it in range(steps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.load_events(*tens, t_end=t_end, validate=False)
        ctx.forward(load, lam, out=P)
        torch.cuda.synchronize()
        if it > 0:
            times.append(time.perf_counter() - t0)
    return 1e3 * sum(times) / len(times)


def forward_record(name, gtp, torch, dev, steps, warmup, adjoint=False, e2w=True, keep=False, **tune):
    """Full-size record of a named configuration: forward rate and its
    roofline fraction (16 B/event), the events-to-waveform rate and,
    optionally, forward + adjoint."""
    import synth
    t0 = time.time()
    prob = synth.make_problem(name)
    gen_s = time.time() - t0
    log(f"generated {name}: {prob.ev.n_events} events in {gen_s:.1f} s")
    ctx, tens, load, lam = open_problem(gtp, torch, dev, prob, **tune)
    P = torch.empty(ctx.n_bins, dtype=torch.float32, device=dev)
    ctx.forward(load, lam, out=P)
    for _ in range(warmup):
        ctx.forward(load, lam, out=P)
    stream = torch.cuda.current_stream(dev)
    ms, kern = timed_forward(ctx, torch, stream, load, lam, P, steps)
    N = prob.ev.n_events
    fwd = kern.get("k_fwd_packed", {}).get("avg_ms")
    rec = {"workload": f"{name}: {WORKLOADS[name]}", "n_events": N, "n_gates": prob.net.n_gates,
           "n_bins": ctx.n_bins, "value": N / (ms * 1e-3), "unit": "events/s", "ms_per_step": ms,
           "k_fwd_packed_ms": fwd, "frac": (EVENT_BYTES * N / (fwd * 1e-3) / HBM_PEAK) if fwd else None,
           "traffic": measured_traffic("k_fwd_packed", name), "pack_ms": ctx.plan_info()["pack_ms"],
           "kernels": kern, "gen_s": gen_s}
    if adjoint:
        ms_fa, kern_fa = timed_fwd_adjoint(ctx, torch, stream, load, lam, P, steps)
        adj = kern_fa.get("k_adjoint_packed", {}).get("avg_ms")
        rec["fwd_adjoint"] = {"value": N / (ms_fa * 1e-3), "unit": "events/s", "ms_per_step": ms_fa,
                              "k_adjoint_packed_ms": adj,
                              "adjoint_frac": (EVENT_BYTES * N / (adj * 1e-3) / HBM_PEAK) if adj else None,
                              "adjoint_traffic": measured_traffic("k_adjoint_packed", name), "kernels": kern_fa}
    if e2w:
        ms_e = events_to_waveform(ctx, torch, tens, prob.ev.t_end, load, lam, P, max(2, min(steps, 3)))
        rec["events_to_waveform"] = {"value": N / (ms_e * 1e-3), "unit": "events/s", "ms_per_step": ms_e,
                                     "pack_ms": ctx.plan_info()["pack_ms"],
                                     "frac": EVENT_BYTES * N / (ms_e * 1e-3) / HBM_PEAK}
    ctx.close()
    out = (rec, prob, P) if keep else rec
    del tens
    return out


def split_comparison(gtp, torch, dev, name, scale, steps):
    """The density-aware packed path against one gate per thread on the same
    (scaled) workload: the longest gate of the full workload alone keeps one
    thread busy far beyond a step, so the comparison runs at `scale`."""
    import synth
    prob = synth.make_problem(name, scale=scale)
    stream = torch.cuda.current_stream(dev)
    res = {}
    for algo in (0, 1):
        ctx, tens, load, lam = open_problem(gtp, torch, dev, prob, algo=algo)
        P = torch.empty(ctx.n_bins, dtype=torch.float32, device=dev)
        ctx.forward(load, lam, out=P)
        ms, _ = timed_forward(ctx, torch, stream, load, lam, P, max(2, min(steps, 5)))
        res[algo] = ms
        ctx.close()
    N = prob.ev.n_events
    return {"scale": scale, "n_events": N, "density_split_ms": res[0], "one_gate_per_thread_ms": res[1],
            "speedup": res[1] / res[0]}


def bench_c4(args, gtp, torch, dev):
    """Batched traces at their full lengths: 64 traces of 10k-1M cycles over
    one 200k-gate netlist, in the fewest trace groups whose events and
    layouts fit the device (each group one persistent batched launch
    replayed from a HIP graph), against one forward per trace."""
    import synth
    lib, net, items, bin_ps = synth.batch_plan(n_traces=args.batch_traces, cycles=tuple(args.batch_cycles))
    free, _ = torch.cuda.mem_get_info(dev)
    budget = int(0.70 * free / BATCH_BYTES_PER_EVENT)   # events per group
    groups, cur, cur_n = [], [], 0
    for it in items:
        if cur and cur_n + it[2] > budget:
            groups.append(cur)
            cur, cur_n = [], 0
        cur.append(it)
        cur_n += it[2]
    groups.append(cur)
    log(f"C4: {sum(it[2] for it in items)} events in {len(groups)} trace groups (budget {budget} events/group)")
    stream = torch.cuda.current_stream(dev)
    steps = max(2, min(args.steps, 5))
    tot_graph = tot_seq = 0.0
    gen_s = plan_s = 0.0
    n_ev = n_bins = 0
    for gi, grp in enumerate(groups):
        t0 = time.time()
        tr = []
        for it in grp:
            ev = synth.batch_trace(lib, net, it)
            tr.append(tuple(torch.from_numpy(a).to(dev) for a in (ev.gate_off, ev.t, ev.pin_bit, ev.slew))
                      + (ev.t_end,))
            del ev
        gen_s += time.time() - t0
        ctx = gtp.Context(0)
        ctx.load_library(lib)
        ctx.load_netlist(torch.from_numpy(net.gate_cell).to(dev), torch.from_numpy(net.gate_out_net).to(dev),
                         torch.from_numpy(net.gate_init.view(np.int32)).to(dev), net.n_nets)
        ctx.set_params(vdd=0.8, bin_ps=bin_ps)
        ctx.load_traces(tr)
        load = torch.from_numpy(net.net_load).to(dev)
        lam = torch.from_numpy(net.leak_scale).to(dev)
        tot, offs = ctx.batch_bins()
        P = torch.empty(tot, dtype=torch.float32, device=dev)
        t1 = time.time()
        ctx.forward_batched(load, lam, out=P, use_graph=True)   # packs every trace, records the graph
        torch.cuda.synchronize()
        plan_s += time.time() - t1
        outs = [P[int(offs[i]):int(offs[i + 1])] for i in range(len(tr))]
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

        def timed(fn):
            fn()
            torch.cuda.synchronize()
            e0.record(stream)
            for _ in range(steps):
                fn()
            e1.record(stream)
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / steps

        def per_trace():
            for i in range(len(tr)):
                ctx.forward_trace(i, load, lam, out=outs[i])

        g_ms = timed(lambda: ctx.forward_batched(load, lam, out=P, use_graph=True))
        s_ms = timed(per_trace)
        tot_graph += g_ms
        tot_seq += s_ms
        n_ev += sum(it[2] for it in grp)
        n_bins += int(tot)
        log(f"C4 group {gi}: {len(grp)} traces, {sum(it[2] for it in grp)} events: graph {g_ms:.2f} ms, "
            f"per-trace {s_ms:.2f} ms")
        ctx.close()
        del tr, P, outs
        torch.cuda.empty_cache()
    cyc = [it[1] // 1000 for it in items]
    return {"workload": f"{len(items)} traces over one {net.n_gates}-gate, {lib.n_cells}-cell netlist, "
                        f"{args.batch_cycles[0]}-{args.batch_cycles[1]} cycles of 1 ns each (drawn), "
                        f"500 events per cycle, lognormal(0,2) per-gate counts, {bin_ps} ps bins",
            "n_events": n_ev, "n_bins": n_bins, "cycles_min": int(min(cyc)), "cycles_max": int(max(cyc)),
            "trace_groups": len(groups), "traces_per_group": [len(g) for g in groups],
            "value": n_ev / (tot_graph * 1e-3), "unit": "events/s", "ms_per_step": tot_graph,
            "per_trace": {"value": n_ev / (tot_seq * 1e-3), "ms_per_step": tot_seq,
                          "launches_per_step": 4 * len(items)},
            "speedup_vs_per_trace": tot_seq / tot_graph, "plan_s": plan_s, "gen_s": gen_s}


def bench_stream(gtp, torch, dev, prob, P_ref, window_cycles):
    """One trace streamed from pinned host memory in windows (gtp_stream_*):
    a helper thread cuts window k+2 out of the host trace while window k+1 is
    copied and window k is evaluated."""
    import concurrent.futures as cf

    import synth
    ev = prob.ev
    T = ev.t_end
    W = window_cycles * 1000
    cuts = list(range(0, T, W)) + [T]
    wins = list(zip(cuts[:-1], cuts[1:]))
    sizes = [synth.window_size(ev, a, b) for a, b in wins]
    cap = max(sizes)
    G = prob.net.n_gates
    bufs = [(torch.empty(G + 1, dtype=torch.int64).pin_memory(), torch.empty(cap, dtype=torch.int64).pin_memory(),
             torch.empty(cap, dtype=torch.uint8).pin_memory(), torch.empty(cap, dtype=torch.float32).pin_memory())
            for _ in range(3)]
    views = [tuple(b.numpy() for b in s) for s in bufs]
    net = prob.net
    ctx = gtp.Context(0)
    ctx.load_library(prob.lib)
    ctx.load_netlist(torch.from_numpy(net.gate_cell).to(dev), torch.from_numpy(net.gate_out_net).to(dev),
                     torch.from_numpy(net.gate_init.view(np.int32)).to(dev), net.n_nets)
    ctx.set_params(vdd=prob.vdd, bin_ps=prob.bin_ps, sw_mode=prob.sw_mode)
    load = torch.from_numpy(net.net_load).to(dev)
    lam = torch.from_numpy(net.leak_scale).to(dev)
    pool = cf.ThreadPoolExecutor(1)

    def run():
        prep = [None] * len(wins)

        def cut(k):
            return synth.window(ev, *wins[k], out=views[k % 3])

        out = ctx.stream_begin(T)
        prep[0] = pool.submit(cut, 0)
        if len(wins) > 1:
            prep[1] = pool.submit(cut, 1)
        prep[0].result()
        ctx.stream_push(*bufs[0][:1], *[b[:sizes[0]] for b in bufs[0][1:]], *wins[0])
        for k in range(len(wins)):
            if k + 1 < len(wins):
                prep[k + 1].result()
                s = bufs[(k + 1) % 3]
                ctx.stream_push(s[0], *[b[:sizes[k + 1]] for b in s[1:]], *wins[k + 1])
            if k + 2 < len(wins):
                prep[k + 2] = pool.submit(cut, k + 2)
            ctx.stream_step(load, lam, out)
        torch.cuda.synchronize()
        ctx.stream_end()
        return out

    run()   # grows the staging buffers and the layout arena
    t0 = time.perf_counter()
    out = run()
    wall = time.perf_counter() - t0
    t0 = time.perf_counter()
    for k in range(len(wins)):
        synth.window(ev, *wins[k], out=views[k % 3])
    cut_s = time.perf_counter() - t0
    pool.shutdown()
    ctx.close()
    d = (out.double() - P_ref.double()).abs() / P_ref.double().abs().clamp_min(1e-30)
    N = ev.n_events
    return {"workload": f"the C3 trace ({N} events, {T // 1000} cycles) in {len(wins)} windows of {window_cycles} "
                        f"cycles from pinned host memory",
            "n_events": N, "windows": len(wins), "max_window_events": cap,
            "value": N / wall, "unit": "events/s", "wall_s": wall, "host_cut_s": cut_s,
            "h2d_bytes": int(sum(sizes) * 13 + len(wins) * (G + 1) * 8),
            "max_rel_diff_vs_in_hbm": float(d.max().item())}


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
    ap.add_argument("--no-configs", action="store_true", help="skip the C3 and C5 records")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-trace (C4) comparison")
    ap.add_argument("--no-stream", action="store_true", help="skip the streamed-window record")
    ap.add_argument("--batch-traces", type=int, default=64)
    ap.add_argument("--batch-cycles", type=int, nargs=2, default=[10_000, 1_000_000],
                    help="range of cycles per trace of the batched comparison")
    ap.add_argument("--stream-window-cycles", type=int, default=25_000)
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
    log(f"generated {args.config}: {prob.ev.n_events} events, {prob.net.n_gates} gates, {prob.n_bins} bins "
        f"in {gen_s:.1f} s")
    net, ev = prob.net, prob.ev
    tp = time.time()
    ctx, tens, load, lam = open_problem(gtp, torch, dev, prob, algo=args.algo, tile_log2=args.tile_log2,
                                        tile_threads=args.tile_threads)
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
    ms_step, kern_avg = timed_forward(ctx, torch, stream, load, lam, P, args.steps)
    N, G, NB = ev.n_events, net.n_gates, ctx.n_bins
    value = N / (ms_step * 1e-3)
    log(f"forward: {ms_step:.3f} ms/step")

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
        # bytes the packed layout actually holds per event: event word, table
        # row and slew weight, unit descriptors, group offsets
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
    if args.algo == 0:
        ms_e2w = events_to_waveform(ctx, torch, tens, ev.t_end, load, lam, P, max(2, min(args.steps, 5)))
        out["events_to_waveform"] = {
            "value": N / (ms_e2w * 1e-3), "unit": "events/s", "ms_per_step": ms_e2w, "pack_ms": ctx.plan_info()["pack_ms"],
            "frac": EVENT_BYTES * N / (ms_e2w * 1e-3) / HBM_PEAK,
            "note": "events in the caller's gate-major layout to FP32 waveform: lane-block plan, packed layout "
                    "(partition, carried-in state, per-event state, table rows, slew weights) and the forward, "
                    "every step"}
        log(f"events to waveform: {ms_e2w:.2f} ms/step")
    # ---- forward + adjoint -------------------------------------------------
    if not args.no_adjoint:
        ms_fa, kern_fa = timed_fwd_adjoint(ctx, torch, stream, load, lam, P, args.steps)
        adj = kern_fa.get("k_adjoint_packed", {}).get("avg_ms")
        out["fwd_adjoint"] = {"value": N / (ms_fa * 1e-3), "unit": "events/s", "ms_per_step": ms_fa,
                              "adjoint_frac": (EVENT_BYTES * N / (adj * 1e-3) / HBM_PEAK) if adj else None,
                              "adjoint_traffic": measured_traffic("k_adjoint_packed", args.config),
                              "kernels": kern_fa}
        log(f"forward + adjoint: {ms_fa:.3f} ms/step")

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
        log(f"cpu baseline: {ns / dt:.3g} events/s")
    ctx.close()
    del tens, prob, P
    torch.cuda.empty_cache()

    # ---- the other configurations at full size -----------------------------
    fsteps = max(2, min(args.steps, 10))
    if not args.no_configs and args.config == "C2" and args.scale == 1.0:
        rec3, prob3, P3 = forward_record("C3", gtp, torch, dev, fsteps, 2, keep=True)
        rec3["vs_one_gate_per_thread"] = split_comparison(gtp, torch, dev, "C3", 0.01, fsteps)
        out["C3"] = rec3
        log(f"C3: {rec3['ms_per_step']:.3f} ms/step")
        if not args.no_stream:
            out["stream"] = bench_stream(gtp, torch, dev, prob3, P3, args.stream_window_cycles)
            log(f"stream: {out['stream']['wall_s']:.2f} s")
        del prob3, P3
        torch.cuda.empty_cache()
        out["C5"] = forward_record("C5", gtp, torch, dev, fsteps, 2, adjoint=True, e2w=False)
        log(f"C5: {out['C5']['ms_per_step']:.3f} ms/step")
    # ---- batched traces: one persistent graph launch per group vs per-trace launches
    if not args.no_batched:
        out["C4"] = bench_c4(args, gtp, torch, dev)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
