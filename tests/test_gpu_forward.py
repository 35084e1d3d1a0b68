"""GPU parity of the forward path against the FP64 oracle, through the C ABI.

Bar: states and bin indices bit-exact; every bin within 1e-5 relative of the
FP64 waveform; both execution paths (packed tile-major, one gate per thread)
give bit-identical FP32 waveforms (exact int64 fixed-point accumulation).
"""
import numpy as np
import pytest

import oracle
import synth
from _problems import build_problem, load_golden, to_device_ctx

pytestmark = pytest.mark.gpu
REL = 1e-5


@pytest.fixture(scope="module")
def O():
    return oracle.get()


def run(prob, algo=0, tile_log2=0):
    ctx, load, lam = to_device_ctx(prob, algo=algo, tile_log2=tile_log2)
    P = ctx.forward(load, lam).cpu().numpy()
    st, b = ctx.event_trace()
    ctx.sync()
    out = P, st.cpu().numpy(), b.cpu().numpy()
    ctx.close()
    return out


def check(prob, O, algos=(0, 1), tile_log2=0):
    P64 = O.power(prob)
    st64, b64 = O.event_trace(prob)
    res = [run(prob, a, tile_log2) for a in algos]
    for P, st, b in res:
        assert np.array_equal(st, st64), "state before group differs"
        assert np.array_equal(b, b64), "bin index differs"
        rel = np.abs(P.astype(np.float64) - P64) / P64
        assert rel.max() <= REL, f"max rel err {rel.max():.3e} at bin {rel.argmax()}"
    for P, _, _ in res[1:]:
        assert np.array_equal(P.view(np.uint32), res[0][0].view(np.uint32)), "paths not bit-identical"
    return res[0][0], P64


@pytest.mark.parametrize("name,mode", [("example_a.json", 0), ("example_a.json", 1), ("example_b.json", 0)])
def test_golden(O, name, mode):
    prob, fx = load_golden(name, sw_mode=mode)
    P, _ = check(prob, O)
    exp = np.asarray(fx["expect"][f"sw_mode_{mode}"]["bins_fj"]) / prob.bin_ps
    np.testing.assert_allclose(P, exp, rtol=REL)


@pytest.mark.parametrize("seed", range(1, 13))
def test_random_small(O, seed):
    rng = np.random.default_rng(seed)
    prob = synth.make_random_small(seed, n_gates=int(rng.integers(1, 60)), n_cells=int(rng.integers(1, 9)),
                                   i_max=int(rng.integers(1, 5)), n_events=int(rng.integers(0, 6000)),
                                   t_end=int(rng.integers(6000, 40000)), bin_ps=int(rng.choice([1, 7, 50, 64, 100, 333])),
                                   p_tie=float(rng.choice([0.0, 0.2, 0.5])), n_clock=int(rng.integers(0, 2)))
    check(prob, O)


@pytest.mark.parametrize("tile_log2", [2, 4, 8, 9, 13])
def test_tile_sizes(O, tile_log2):
    prob = synth.make_random_small(21, n_gates=200, n_cells=8, i_max=4, n_events=30000, t_end=200000, bin_ps=10,
                                   p_tie=0.1, n_clock=3)
    check(prob, O, algos=(0,), tile_log2=tile_log2)


def test_c1(O):
    """Parity configuration: 1k gates, 8 cells, 100k events, 100 ps bins."""
    prob = synth.make_problem("C1")
    check(prob, O)


def test_partial_last_bin_and_edges(O):
    """t_end not a multiple of the bin width; events at 0, bin boundaries, t_end-1."""
    cell = dict(n_inputs=2, slew_axis=[5.0, 50.0, 500.0], load_axis=[0.5, 5.0, 50.0], leak=[3.0, 9.0, 27.0, 1.0],
                table_fn=lambda s, d: np.arange(9, dtype=float).reshape(3, 3) * (1 + s) + d)
    T = 1050
    ev = [(0, 0, 0, 1, 1.0), (0, 100, 1, 1, 600.0), (0, 100, 2, 1, 5.0), (0, 199, 0, 0, 50.0), (0, 200, 2, 0, 500.0),
          (0, T - 1, 1, 0, 0.5), (1, 1000, 0, 1, 20.0), (1, 1049, 1, 1, 20.0)]
    prob = build_problem([cell], [dict(cell=0, init=[0, 0, 0], load=50.0, leak_scale=1.5),
                                  dict(cell=0, init=[0, 0, 1], load=0.25, leak_scale=0.0)], ev, T, 100)
    check(prob, O)


def test_empty_and_sparse(O):
    """No events at all; gates without events between busy ones; a ragged tail."""
    lib = synth.make_library(3, 4, 3)
    net = synth.make_netlist(3, lib, 50)
    ev = synth.Events(0, 5000, np.zeros(51, np.int64), np.zeros(0, np.int64), np.zeros(0, np.uint8),
                      np.zeros(0, np.float32))
    check(synth.Problem(lib, net, ev, vdd=0.8, bin_ps=100), O)
    counts = np.zeros(50, np.int64)
    counts[[0, 7, 8, 30, 49]] = [3, 1, 40, 17, 5]
    is_clock = np.zeros(50, np.uint8)
    ev2 = synth.make_events(3, lib, net, counts, is_clock, 5000, 1000, p_tie=0.3)
    check(synth.Problem(lib, net, ev2, vdd=0.8, bin_ps=100), O)


def test_dense_single_gate(O):
    """One gate holding every event (a dense gate cut across many lane blocks and tiles)."""
    lib = synth.make_library(4, 2, 4)
    net = synth.make_netlist(4, lib, 3)
    counts = np.array([0, 50003, 0], np.int64)
    ev = synth.make_events(4, lib, net, counts, np.zeros(3, np.uint8), 100000, 1000, p_tie=0.4)
    check(synth.Problem(lib, net, ev, vdd=0.8, bin_ps=5), O)


def test_sw_mode_paper(O):
    prob = synth.make_random_small(31, n_gates=30, n_events=3000)
    prob.sw_mode = 1
    check(prob, O)


def test_run_to_run_identical(O):
    prob = synth.make_problem("C1", scale=0.5)
    a = run(prob)[0]
    b = run(prob)[0]
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))


def test_plan_invariants(O):
    """Every in-window event is packed exactly once, units hold at most 16
    events, groups hold at most 64 units, and the packed trace covers every
    event (checked against the oracle in check())."""
    prob = synth.make_random_small(41, n_gates=300, n_cells=8, i_max=4, n_events=60000, t_end=500000, bin_ps=50,
                                   p_tie=0.2, n_clock=4)
    ctx, load, lam = to_device_ctx(prob, algo=0)
    info = ctx.plan_info()
    ctx.close()
    N = prob.ev.n_events
    assert info["n_events_packed"] == N
    assert -(-N // 16) <= info["n_units"] <= N
    assert -(-info["n_units"] // 64) <= info["n_groups"] <= -(-info["n_units"] // 64) + info["n_tiles"]
    assert info["n_tiles"] == -(-prob.n_bins // (1 << info["tile_log2"]))
    check(prob, O)


def test_wide_bins_fixed_point_range(O):
    """Bins of 2^22 ps holding 10^6 events each (about 10^7 fJ per bin, beyond
    the 2^23 fJ an energy unit of 2^-40 fJ allows in int64): the library picks
    a coarser unit from its range bounds, and every bin still matches the
    oracle within 1e-5 (a wrapped accumulator would be off by 2^63 units)."""
    lib = synth.make_library(12, 4, 4)
    net = synth.make_netlist(12, lib, 16)
    counts = np.full(16, 125000, np.int64)
    ev = synth.make_events(12, lib, net, counts, np.zeros(16, np.uint8), 1 << 23, 1000, p_tie=0.1)
    prob = synth.Problem(lib, net, ev, vdd=0.8, bin_ps=1 << 22)
    P, P64 = check(prob, O)
    assert (P64 * prob.bin_ps).max() > 2.0 ** 23   # the per-bin energy the unit 2^-40 fJ cannot hold


def test_table_order_independent_of_cell_order(O):
    """Cells whose table blocks are stored in the reverse of the cell order
    (the library's table bases need not grow with the cell index): the
    waveform equals the oracle's and, bit for bit, the one of the same library
    stored in cell order."""
    import dataclasses
    prob = synth.make_problem("C1")
    lib = prob.lib
    per = lib.n_slew * lib.n_load
    n_tab = lib.tables.size // per
    ends = list(lib.table_base[1:]) + [n_tab]
    blocks = [lib.tables[b * per:e * per] for b, e in zip(lib.table_base, ends)]
    base, pos = np.zeros(lib.n_cells, np.int64), 0
    for c in reversed(range(lib.n_cells)):
        base[c] = pos
        pos += blocks[c].size // per
    tables = np.concatenate([blocks[c] for c in reversed(range(lib.n_cells))])
    prob2 = dataclasses.replace(prob, lib=dataclasses.replace(lib, table_base=base, tables=tables))
    P_ref, _ = check(prob, O)
    P_rev, _ = check(prob2, O)
    assert np.array_equal(P_ref.view(np.uint32), P_rev.view(np.uint32))
