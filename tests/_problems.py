"""Hand-specified problems (golden fixtures, brute-force cases) as synth.Problem."""
import json
import os

import numpy as np

import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def build_problem(cells, gates, events, t_end, bin_ps, vdd=0.8, sw_mode=0, extra_nets=0):
    """cells: list of dict(n_inputs, slew_axis, load_axis, leak, tables{"s,d": 2D list} or table_fn(s,d)->2D).
    gates: list of dict(cell, init (list of pin values, output last) or init_bits, load, leak_scale).
    events: list of (gate, t, pin, value, slew); will be stably sorted gate-major by time."""
    n_cells = len(cells)
    n_slew = len(cells[0]["slew_axis"])
    n_load = len(cells[0]["load_axis"])
    n_inputs = np.array([c["n_inputs"] for c in cells], np.int32)
    slew_axis = np.concatenate([np.asarray(c["slew_axis"], np.float32) for c in cells])
    load_axis = np.concatenate([np.asarray(c["load_axis"], np.float32) for c in cells])
    map_base, s2t, table_base, tables, leak_base, leak = [], [], [], [], [], []
    mb = tb = lb = 0
    for c in cells:
        ns = 1 << c["n_inputs"]
        map_base.append(mb); table_base.append(tb); leak_base.append(lb)
        for s in range(ns):
            for d in range(2):
                s2t.append(2 * s + d)
                if "tables" in c:
                    T = np.asarray(c["tables"][f"{s},{d}"], np.float64)
                else:
                    T = np.asarray(c["table_fn"](s, d), np.float64)
                assert T.shape == (n_slew, n_load)
                tables.append(T.astype(np.float32).ravel())
        leak.extend(np.asarray(c["leak"], np.float32).tolist())
        mb += 2 * ns; tb += 2 * ns; lb += ns
    lib = synth.Library(n_cells, n_slew, n_load, n_inputs, slew_axis, load_axis,
                        np.array(map_base, np.int64), np.array(s2t, np.int16), np.array(table_base, np.int64),
                        np.concatenate(tables).astype(np.float32), np.array(leak_base, np.int64),
                        np.array(leak, np.float32))
    G = len(gates)
    gate_cell = np.array([g["cell"] for g in gates], np.int32)
    init = []
    for g in gates:
        if "init_bits" in g:
            init.append(int(g["init_bits"]))
        else:
            init.append(sum(int(v) << p for p, v in enumerate(g["init"])))
    n_nets = G + extra_nets
    gate_out = np.arange(extra_nets, extra_nets + G, dtype=np.int32)
    net_load = np.full(n_nets, 1.0, np.float32)
    net_load[gate_out] = [g["load"] for g in gates]
    net = synth.Netlist(G, n_nets, gate_cell, gate_out, np.array(init, np.uint32), net_load,
                        np.array([g.get("leak_scale", 1.0) for g in gates], np.float32))
    ev = sorted(((int(e[0]), int(e[1]), k, e) for k, e in enumerate(events)))
    counts = np.zeros(G, np.int64)
    for e in ev:
        counts[e[0]] += 1
    gate_off = np.zeros(G + 1, np.int64)
    np.cumsum(counts, out=gate_off[1:])
    t = np.array([e[3][1] for e in ev], np.int64)
    pin_bit = np.array([(int(e[3][2]) << 1) | int(e[3][3]) for e in ev], np.uint8)
    slew = np.array([e[3][4] for e in ev], np.float32)
    events_ = synth.Events(len(ev), int(t_end), gate_off, t, pin_bit, slew)
    return synth.Problem(lib, net, events_, vdd=vdd, bin_ps=int(bin_ps), sw_mode=sw_mode, name="hand")


def load_golden(name, sw_mode=0):
    with open(os.path.join(GOLDEN, name)) as f:
        fx = json.load(f)
    prob = build_problem(fx["cells"], fx["gates"], fx["events"], fx["t_end"], fx["bin_ps"], fx["vdd"], sw_mode)
    prob.glitch_clk = int(fx.get("glitch_clk", 0))
    return prob, fx


def to_device_ctx(prob, algo=0, tile_log2=0, validate=True):
    """Load a synth.Problem into a library Context on cuda:0; returns
    (ctx, net_load, leak_scale) with the loads and scales on the device."""
    import torch

    import paper_2609_05960_amd as gtp

    dev = torch.device("cuda", 0)
    ctx = gtp.Context(0)
    ctx.load_library(prob.lib, all_pin_state=int(getattr(prob, "state_all_pins", 0)))
    net, ev = prob.net, prob.ev
    ctx.load_netlist(torch.from_numpy(net.gate_cell).to(dev), torch.from_numpy(net.gate_out_net).to(dev),
                     torch.from_numpy(net.gate_init.view(np.int32)).to(dev), net.n_nets)
    tens = [torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in (ev.gate_off, ev.t, ev.pin_bit, ev.slew)]
    ctx.load_events(*tens, t_end=ev.t_end, validate=validate)
    ctx.set_params(vdd=prob.vdd, bin_ps=prob.bin_ps, sw_mode=prob.sw_mode,
                   glitch_clk_ps=int(getattr(prob, "glitch_clk", 0)))
    ctx.set_tuning(algo=algo, bins_per_tile_log2=tile_log2)
    load = torch.from_numpy(net.net_load).to(dev)
    lam = torch.from_numpy(net.leak_scale).to(dev)
    return ctx, load, lam


def all_pin_library(lib, seed=0):
    """The library re-indexed over every pin (bit I = the output): the output
    value selects a different table and scales the leakage, so the state the
    output holds matters (same construction as the oracle pins use)."""
    rng = np.random.default_rng(seed)
    map_base, s2t, leak_base, leak = [], [], [], []
    for c in range(lib.n_cells):
        I = int(lib.n_inputs[c])
        n_tab = 2 << I
        map_base.append(len(s2t))
        leak_base.append(len(leak))
        for s in range(2 << I):
            si, out = s & ((1 << I) - 1), s >> I
            for d in range(2):
                k = int(lib.state_to_table[lib.map_base[c] + 2 * si + d])
                s2t.append(k if out == 0 else (k + 1) % n_tab)
            leak.append(float(lib.leak[lib.leak_base[c] + si]) * (1.0 + out * float(rng.uniform(0.2, 1.0))))
    return synth.Library(lib.n_cells, lib.n_slew, lib.n_load, lib.n_inputs, lib.slew_axis, lib.load_axis,
                         np.array(map_base, np.int64), np.array(s2t, np.int16), lib.table_base, lib.tables,
                         np.array(leak_base, np.int64), np.array(leak, np.float32))
