"""Seeded synthetic workloads (inputs only; no power arithmetic).

Builds a cell library, a netlist and gate-major toggle-event streams with the
shapes of the paper's workloads (Sec. 6.1 designs, Sec. 3.2 heavy-tailed
per-gate event counts) at the sizes of the named configurations below.
Both the FP64 reference evaluator and the GPU library consume these arrays.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libsynth.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile libsynth.so in-tree (gcc, OpenMP)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp,
                               os.path.join(_HERE, "synth.c"), "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        _lib = ctypes.CDLL(_SO)
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _check(rc: int, what: str):
    if rc != 0:
        raise RuntimeError(f"synth: {what} failed with code {rc}")


@dataclasses.dataclass
class Library:
    n_cells: int
    n_slew: int
    n_load: int
    n_inputs: np.ndarray        # int32 [n_cells]
    slew_axis: np.ndarray       # float32 [n_cells*n_slew] ps
    load_axis: np.ndarray       # float32 [n_cells*n_load] fF
    map_base: np.ndarray        # int64 [n_cells] -> first int16 of the cell's [2^I][2] map
    state_to_table: np.ndarray  # int16: local table id per (state, dir)
    table_base: np.ndarray      # int64 [n_cells] -> first table of the cell
    tables: np.ndarray          # float32 [n_tables*n_slew*n_load] fJ, [table][slew][load]
    leak_base: np.ndarray       # int64 [n_cells]
    leak: np.ndarray            # float32 nW, [2^I] per cell
    # optional state patterns (a cell with n_tpat[c] > 0 is given by them)
    n_tpat: Optional[np.ndarray] = None      # int32 [n_cells]
    tpat_base: Optional[np.ndarray] = None   # int64 [n_cells]
    tpat_care: Optional[np.ndarray] = None   # uint32, bit p = pin p named by the pattern
    tpat_value: Optional[np.ndarray] = None  # uint32, values of the named pins
    tpat_table: Optional[np.ndarray] = None  # int16 [2 * patterns]: local table id (fall, rise)
    n_lpat: Optional[np.ndarray] = None
    lpat_base: Optional[np.ndarray] = None
    lpat_care: Optional[np.ndarray] = None
    lpat_value: Optional[np.ndarray] = None
    lpat_leak: Optional[np.ndarray] = None   # float32 nW


@dataclasses.dataclass
class Netlist:
    n_gates: int
    n_nets: int
    gate_cell: np.ndarray       # int32 [G]
    gate_out_net: np.ndarray    # int32 [G]
    gate_init: np.ndarray       # uint32 [G], bit p = initial value of pin p (output = pin I)
    net_load: np.ndarray        # float32 [n_nets] fF
    leak_scale: np.ndarray      # float32 [G]


@dataclasses.dataclass
class Events:
    n_events: int
    t_end: int
    gate_off: np.ndarray        # int64 [G+1]
    t: np.ndarray               # int64 [N] ps
    pin_bit: np.ndarray         # uint8 [N] (pin<<1)|new_value
    slew: np.ndarray            # float32 [N] ps


@dataclasses.dataclass
class Problem:
    lib: Library
    net: Netlist
    ev: Events
    vdd: float
    bin_ps: int
    sw_mode: int = 0
    name: str = ""
    state_all_pins: int = 0     # 1: state index over every pin (bit I = output); the library then holds 2^(I+1) states
    glitch_clk: int = 0         # clock period of the glitch detection (ps); 0: off

    @property
    def n_bins(self) -> int:
        return -(-self.ev.t_end // self.bin_ps)


def make_library(seed: int, n_cells: int, i_max: int, n_slew: int = 7, n_load: int = 7,
                 slew_range=(5.0, 500.0), load_range=(0.5, 50.0), leak_range=(1.0, 50.0)) -> Library:
    L = _load()
    n_inputs = np.zeros(n_cells, np.int32)
    _check(L.synth_cell_inputs(ctypes.c_uint64(seed), ctypes.c_int32(n_cells), ctypes.c_int32(i_max),
                               _p(n_inputs)), "cell_inputs")
    ns = (1 << n_inputs.astype(np.int64))
    n_map = int((2 * ns).sum())
    n_tab = int((2 * ns).sum())
    n_leak = int(ns.sum())
    slew_axis = np.zeros(n_cells * n_slew, np.float32)
    load_axis = np.zeros(n_cells * n_load, np.float32)
    map_base = np.zeros(n_cells, np.int64)
    s2t = np.zeros(n_map, np.int16)
    table_base = np.zeros(n_cells, np.int64)
    tables = np.zeros(n_tab * n_slew * n_load, np.float32)
    leak_base = np.zeros(n_cells, np.int64)
    leak = np.zeros(n_leak, np.float32)
    d = ctypes.c_double
    _check(L.synth_library(ctypes.c_uint64(seed), ctypes.c_int32(n_cells), ctypes.c_int32(n_slew),
                           ctypes.c_int32(n_load), _p(n_inputs), d(slew_range[0]), d(slew_range[1]),
                           d(load_range[0]), d(load_range[1]), d(leak_range[0]), d(leak_range[1]),
                           _p(slew_axis), _p(load_axis), _p(map_base), _p(s2t), _p(table_base), _p(tables),
                           _p(leak_base), _p(leak)), "library")
    return Library(n_cells, n_slew, n_load, n_inputs, slew_axis, load_axis, map_base, s2t, table_base,
                   tables, leak_base, leak)


def add_pattern_cells(lib: Library, seed: int, wide_inputs=(), convert=(), all_pins: int = 0,
                      n_pat=(2, 12), max_care: int = 4, leak_range=(1.0, 50.0)) -> Library:
    """A copy of `lib` with cells given by state patterns: new cells with the
    input counts in `wide_inputs` (appended, up to 31 inputs) and the existing
    cells listed in `convert` (their per-state arrays stay but are unused).
    Each cell gets 1 + U{n_pat} table patterns and as many leakage patterns
    drawn the same way: every pattern but the last names 1..max_care random
    state pins (value bits are random on every pin, named or not), the last
    names none (the default). Table pattern k selects two new tables of the
    cell (fall, rise), with entries of the same family as make_library's;
    leakage values ~ U(leak_range) nW. numpy generator seeded with `seed`."""
    rng = np.random.default_rng(seed)
    ns, nl = lib.n_slew, lib.n_load
    n_old = lib.n_cells
    n_cells = n_old + len(wide_inputs)
    n_inputs = np.concatenate([lib.n_inputs, np.asarray(wide_inputs, np.int32)]).astype(np.int32)
    slew_axis = np.concatenate([lib.slew_axis] + [lib.slew_axis[:ns]] * len(wide_inputs)).astype(np.float32)
    load_axis = np.concatenate([lib.load_axis] + [lib.load_axis[:nl]] * len(wide_inputs)).astype(np.float32)
    map_base = np.concatenate([lib.map_base, np.zeros(len(wide_inputs), np.int64)])
    leak_base = np.concatenate([lib.leak_base, np.zeros(len(wide_inputs), np.int64)])
    table_base = np.concatenate([lib.table_base, np.zeros(len(wide_inputs), np.int64)])
    tables = [lib.tables]
    n_tab = lib.tables.size // (ns * nl)
    n_tpat = np.zeros(n_cells, np.int32)
    n_lpat = np.zeros(n_cells, np.int32)
    tpat_base = np.zeros(n_cells, np.int64)
    lpat_base = np.zeros(n_cells, np.int64)
    tc, tv, tt, lc, lv, ll = [], [], [], [], [], []
    patterned = list(convert) + list(range(n_old, n_cells))

    def patterns(nsp, n):
        care, value = [], []
        for k in range(n):
            c = 0
            if k + 1 < n:
                m = int(rng.integers(1, min(max_care, nsp) + 1))
                for p in rng.choice(nsp, size=m, replace=False):
                    c |= 1 << int(p)
            care.append(c)
            value.append(int(rng.integers(0, 1 << 32, dtype=np.uint64)) & 0xffffffff)
        return care, value

    for c in patterned:
        nsp = int(n_inputs[c]) + all_pins
        nt = 1 + int(rng.integers(n_pat[0], n_pat[1] + 1))
        nlp = 1 + int(rng.integers(n_pat[0], n_pat[1] + 1))
        tpat_base[c], lpat_base[c] = len(tc), len(lc)
        n_tpat[c], n_lpat[c] = nt, nlp
        care, value = patterns(nsp, nt)
        tc += care
        tv += value
        tt += list(range(2 * nt))
        care, value = patterns(nsp, nlp)
        lc += care
        lv += value
        ll += list(rng.uniform(*leak_range, nlp))
        table_base[c] = n_tab
        sv = slew_axis[c * ns:(c + 1) * ns].astype(np.float64)[:, None] / 100.0
        cv = load_axis[c * nl:(c + 1) * nl].astype(np.float64)[None, :] / 10.0
        for _ in range(2 * nt):
            e = rng.uniform(0.05, 2.0, 4)
            tables.append((e[0] + e[1] * sv + e[2] * cv + e[3] * np.sqrt(sv * cv)).astype(np.float32).ravel())
        n_tab += 2 * nt
    return Library(n_cells, ns, nl, n_inputs, slew_axis, load_axis, map_base, lib.state_to_table, table_base,
                   np.concatenate(tables).astype(np.float32), leak_base, lib.leak,
                   n_tpat=n_tpat, tpat_base=tpat_base, tpat_care=np.asarray(tc, np.uint32),
                   tpat_value=np.asarray(tv, np.uint32), tpat_table=np.asarray(tt, np.int16), n_lpat=n_lpat,
                   lpat_base=lpat_base, lpat_care=np.asarray(lc, np.uint32), lpat_value=np.asarray(lv, np.uint32),
                   lpat_leak=np.asarray(ll, np.float32))


def make_netlist(seed: int, lib: Library, n_gates: int, load_range=(0.5, 50.0), n_pi: Optional[int] = None) -> Netlist:
    L = _load()
    if n_pi is None:
        n_pi = max(32, n_gates // 100)
    n_nets = n_pi + n_gates
    gate_cell = np.zeros(n_gates, np.int32)
    gate_out = np.zeros(n_gates, np.int32)
    gate_init = np.zeros(n_gates, np.uint32)
    net_load = np.zeros(n_nets, np.float32)
    _check(L.synth_netlist(ctypes.c_uint64(seed), ctypes.c_int64(n_gates), ctypes.c_int32(lib.n_cells),
                           _p(lib.n_inputs), ctypes.c_int64(n_pi), ctypes.c_double(load_range[0]),
                           ctypes.c_double(load_range[1]), _p(gate_cell), _p(gate_out), _p(gate_init),
                           _p(net_load)), "netlist")
    return Netlist(n_gates, n_nets, gate_cell, gate_out, gate_init, net_load, np.ones(n_gates, np.float32))


def make_counts(seed: int, n_gates: int, n_clock: int, clock_events: int, dist: str, p1: float, p2: float,
                total_other: int, max_per_gate: int):
    L = _load()
    is_clock = np.zeros(n_gates, np.uint8)
    _check(L.synth_is_clock(ctypes.c_int64(n_gates), ctypes.c_int64(n_clock), _p(is_clock)), "is_clock")
    counts = np.zeros(n_gates, np.int64)
    dcode = {"lognormal": 0, "zipf": 1, "uniform": 2}[dist]
    _check(L.synth_counts(ctypes.c_uint64(seed), ctypes.c_int64(n_gates), _p(is_clock),
                          ctypes.c_int64(clock_events), ctypes.c_int32(dcode), ctypes.c_double(p1),
                          ctypes.c_double(p2), ctypes.c_int64(total_other), ctypes.c_int64(max_per_gate),
                          _p(counts)), "counts")
    return counts, is_clock


def make_events(seed: int, lib: Library, net: Netlist, counts: np.ndarray, is_clock: np.ndarray, t_end: int,
                t_clk: int, p_tie: float = 0.0, slew_range=(5.0, 500.0)) -> Events:
    L = _load()
    G = net.n_gates
    gate_off = np.zeros(G + 1, np.int64)
    np.cumsum(counts, out=gate_off[1:])
    N = int(gate_off[-1])
    t = np.empty(N, np.int64)
    pin_bit = np.empty(N, np.uint8)
    slew = np.empty(N, np.float32)
    _check(L.synth_events(ctypes.c_uint64(seed), ctypes.c_int64(G), _p(net.gate_cell), _p(lib.n_inputs),
                          _p(net.gate_init), _p(is_clock), _p(gate_off), ctypes.c_int64(t_end),
                          ctypes.c_int64(t_clk), ctypes.c_double(p_tie), ctypes.c_double(slew_range[0]),
                          ctypes.c_double(slew_range[1]), _p(t), _p(pin_bit), _p(slew)), "events")
    return Events(N, t_end, gate_off, t, pin_bit, slew)


def window_size(ev: Events, t0: int, t1: int) -> int:
    """Number of events of ev with t0 <= t < t1."""
    L = _load()
    G = len(ev.gate_off) - 1
    off = np.empty(G + 1, np.int64)
    n = ctypes.c_int64()
    _check(L.synth_window(ctypes.c_int64(G), _p(ev.gate_off), _p(ev.t), _p(ev.pin_bit), _p(ev.slew),
                          ctypes.c_int64(t0), ctypes.c_int64(t1), _p(off), None, None, None, ctypes.byref(n)),
           "window count")
    return n.value


def window(ev: Events, t0: int, t1: int, out=None):
    """The events of ev with t0 <= t < t1 as a gate-major CSR (absolute
    times): (gate_off, t, pin_bit, slew). `out` may give the four arrays to
    fill (e.g. views of pinned buffers, each large enough); the returned
    arrays are then views of them."""
    L = _load()
    G = len(ev.gate_off) - 1
    off = np.empty(G + 1, np.int64) if out is None else out[0][:G + 1]
    n = ctypes.c_int64()
    _check(L.synth_window(ctypes.c_int64(G), _p(ev.gate_off), _p(ev.t), _p(ev.pin_bit), _p(ev.slew),
                          ctypes.c_int64(t0), ctypes.c_int64(t1), _p(off), None, None, None, ctypes.byref(n)),
           "window count")
    m = n.value
    if out is None:
        t, pb, sl = np.empty(m, np.int64), np.empty(m, np.uint8), np.empty(m, np.float32)
    else:
        t, pb, sl = out[1][:m], out[2][:m], out[3][:m]
    _check(L.synth_window(ctypes.c_int64(G), _p(ev.gate_off), _p(ev.t), _p(ev.pin_bit), _p(ev.slew),
                          ctypes.c_int64(t0), ctypes.c_int64(t1), _p(off), _p(t), _p(pb), _p(sl), ctypes.byref(n)),
           "window")
    return off, t, pb, sl


# Named configurations (sizes of the synthetic workloads; recipe in the design doc).
CONFIGS = {
    # 1k gates, 8 cells (1-3 inputs), 100k events over 1,000 cycles of 1 ns,
    # lognormal(3,1.5) counts, 1% clock gates toggling every half cycle, 100 ps bins.
    "C1": dict(seed=1, n_gates=1000, n_cells=8, i_max=3, n_cyc=1000, t_clk=1000, bin_ps=100,
               load_range=(0.5, 20.0), n_clock=10, dist="lognormal", p1=3.0, p2=1.5, total=100_000),
    # 1M gates, 64 cells (1-4 inputs), 200M events over 100k cycles, 50 ps bins,
    # lognormal(4,2) counts, 200 clock gates (clock share 20% of events as in C1).
    "C2": dict(seed=2, n_gates=1_000_000, n_cells=64, i_max=4, n_cyc=100_000, t_clk=1000, bin_ps=50,
               load_range=(0.5, 50.0), n_clock=200, dist="lognormal", p1=4.0, p2=2.0, total=200_000_000),
    # 5M gates, 64 cells, 1B events, Zipf(1.2) counts, 200k cycles, 100 ps bins.
    "C3": dict(seed=3, n_gates=5_000_000, n_cells=64, i_max=4, n_cyc=200_000, t_clk=1000, bin_ps=100,
               load_range=(0.5, 50.0), n_clock=0, dist="zipf", p1=1.2, p2=0.0, total=1_000_000_000),
    # 1M gates, 64 cells, 100M events over 50k cycles, 50 ps bins (adjoint workload).
    "C5": dict(seed=5, n_gates=1_000_000, n_cells=64, i_max=4, n_cyc=50_000, t_clk=1000, bin_ps=50,
               load_range=(0.5, 50.0), n_clock=0, dist="lognormal", p1=4.0, p2=2.0, total=100_000_000),
}


def make_problem(name: str = "C1", scale: float = 1.0, p_tie: float = 0.0, **over) -> Problem:
    """Build a named configuration. `scale` shrinks gates, cycles and events
    together (for tests); overrides replace individual recipe fields."""
    cfg = dict(CONFIGS[name])
    cfg.update(over)
    G = max(1, int(round(cfg["n_gates"] * scale)))
    n_cyc = max(1, int(round(cfg["n_cyc"] * scale)))
    total = int(round(cfg["total"] * scale))
    n_clock = int(round(cfg["n_clock"] * scale)) if cfg["n_clock"] else 0
    t_end = n_cyc * cfg["t_clk"]
    seed = cfg["seed"]
    lib = make_library(seed, cfg["n_cells"], cfg["i_max"], load_range=(0.5, 50.0))
    net = make_netlist(seed, lib, G, load_range=cfg["load_range"])
    clock_events = 2 * n_cyc - 1
    counts, is_clock = make_counts(seed, G, n_clock, clock_events, cfg["dist"], cfg["p1"], cfg["p2"],
                                   total - n_clock * clock_events, t_end)
    ev = make_events(seed, lib, net, counts, is_clock, t_end, cfg["t_clk"], p_tie=p_tie)
    return Problem(lib, net, ev, vdd=0.8, bin_ps=cfg["bin_ps"], sw_mode=0, name=name)


def batch_plan(n_traces: int = 64, cycles=(10_000, 1_000_000), events_per_cycle: int = 500, n_gates: int = 200_000,
               n_cells: int = 32, i_max: int = 4, t_clk: int = 1000, bin_ps: int = 50, seed: int = 4):
    """The batched workload of make_batch without generating its traces:
    (library, netlist, [(trace seed, t_end, events)], bin_ps); batch_trace
    generates one trace of it (the same arrays make_batch returns)."""
    L = _load()
    lib = make_library(seed, n_cells, i_max, load_range=(0.5, 50.0))
    net = make_netlist(seed, lib, n_gates, load_range=(0.5, 50.0))
    draws = np.zeros(n_traces, np.uint64)
    _check(L.synth_draws(ctypes.c_uint64(seed), ctypes.c_uint64(4), ctypes.c_uint64(0), ctypes.c_int64(n_traces),
                         _p(draws)), "draws")
    lo, hi = int(cycles[0]), int(cycles[1])
    items = []
    for i in range(n_traces):
        n_cyc = lo + int(draws[i] % np.uint64(hi - lo + 1))
        items.append((seed * 1_000_003 + i + 1, n_cyc * t_clk, events_per_cycle * n_cyc))
    return lib, net, items, bin_ps


def batch_trace(lib: Library, net: Netlist, item, t_clk: int = 1000, p_tie: float = 0.0) -> Events:
    tseed, t_end, total = item
    counts, is_clock = make_counts(tseed, net.n_gates, 0, 0, "lognormal", 0.0, 2.0, total, t_end)
    return make_events(tseed, lib, net, counts, is_clock, t_end, t_clk, p_tie=p_tie)


def make_batch(n_traces: int = 64, cycles=(10_000, 1_000_000), events_per_cycle: int = 500, n_gates: int = 200_000,
               n_cells: int = 32, i_max: int = 4, t_clk: int = 1000, bin_ps: int = 50, seed: int = 4,
               p_tie: float = 0.0):
    """Batched workload: one netlist and n_traces stimulus traces of uneven
    length. Trace i runs N_cyc,i cycles, N_cyc,i drawn uniformly from `cycles`
    (counter stream 4, index i), with events_per_cycle * N_cyc,i events whose
    per-gate counts follow lognormal(0, 2) weights redrawn per trace; no clock
    gates. Returns (library, netlist, [Events], bin_ps)."""
    lib, net, items, bin_ps = batch_plan(n_traces, cycles, events_per_cycle, n_gates, n_cells, i_max, t_clk, bin_ps,
                                         seed)
    return lib, net, [batch_trace(lib, net, it, t_clk, p_tie) for it in items], bin_ps


def make_random_small(seed: int, n_gates: int = 20, n_cells: int = 4, i_max: int = 3, n_events: int = 400,
                      t_end: int = 5000, bin_ps: int = 100, p_tie: float = 0.2, n_clock: int = 0,
                      dist: str = "lognormal", n_slew: int = 7, n_load: int = 7, vdd: float = 0.8,
                      leak_scale_range=(0.5, 2.0)) -> Problem:
    """Small random problem for parity tests (ties, random leak scales)."""
    lib = make_library(seed, n_cells, i_max, n_slew=n_slew, n_load=n_load)
    net = make_netlist(seed, lib, n_gates, load_range=(0.5, 50.0))
    rng = np.random.default_rng(seed)
    net.leak_scale = rng.uniform(*leak_scale_range, n_gates).astype(np.float32)
    t_clk = 1000
    clock_events = max(0, 2 * (t_end // t_clk) - 1)
    counts, is_clock = make_counts(seed, n_gates, n_clock, clock_events, dist, 1.0, 1.0,
                                   n_events - n_clock * clock_events, t_end)
    ev = make_events(seed, lib, net, counts, is_clock, t_end, t_clk, p_tie=p_tie)
    return Problem(lib, net, ev, vdd=vdd, bin_ps=bin_ps, sw_mode=0, name=f"rand{seed}")
