"""Sort-key widths of the layout builder.

The unit sort key holds (tile, gate block, length class, gate index within
the block). It is 24 bits wide when the first three fields leave room (the
gate index then shifted, its whole value carried by the unit's first event
record), else at most 30 bits (sorted in three passes of 10-bit digits), else
32 bits, else 64 bits with every field whole. The workloads of the other tests
use 24-bit keys; these problems force the wider ones (many
4-bin tiles, small gate blocks, 16-event units) and check every bin against
the FP64 oracle, every event's state and bin bit for bit, and the packed path
against one gate per thread bit for bit.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
REL = 1e-5


@pytest.fixture(scope="module")
def O():
    return oracle.get()


def run(prob, algo, **tune):
    import torch

    import paper_2609_05960_amd as gtp

    dev = torch.device("cuda", 0)
    ctx = gtp.Context(0)
    ctx.load_library(prob.lib)
    net, ev = prob.net, prob.ev
    ctx.load_netlist(torch.from_numpy(net.gate_cell).to(dev), torch.from_numpy(net.gate_out_net).to(dev),
                     torch.from_numpy(net.gate_init.view(np.int32)).to(dev), net.n_nets)
    tens = [torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in (ev.gate_off, ev.t, ev.pin_bit, ev.slew)]
    ctx.load_events(*tens, t_end=ev.t_end, validate=True)
    ctx.set_params(vdd=prob.vdd, bin_ps=prob.bin_ps, sw_mode=prob.sw_mode)
    ctx.set_tuning(algo=algo, **tune)
    P = ctx.forward(torch.from_numpy(net.net_load).to(dev), torch.from_numpy(net.leak_scale).to(dev)).cpu().numpy()
    st, b = ctx.event_trace()
    out = P, st.cpu().numpy(), b.cpu().numpy()
    ctx.close()
    return out


@pytest.mark.parametrize("case", ["key32", "key64"])
def test_wide_sort_keys(O, case):
    if case == "key32":
        # 2^16 tiles (16 bits), 64 one-block cells (6), 8-event units (3): 25 bits, a 30-bit key
        prob = synth.make_random_small(71, n_gates=512, n_cells=64, i_max=3, n_events=60000, t_end=1 << 19,
                                       bin_ps=2, p_tie=0.1, n_clock=2)
        tune = dict(bins_per_tile_log2=2, tile_threads=256)
    else:
        # 2^22 tiles (22 bits), about 128 blocks of 64 gates (7-8), 16-event units (4): more than 32 bits
        prob = synth.make_random_small(72, n_gates=8192, n_cells=64, i_max=3, n_events=80000, t_end=1 << 25,
                                       bin_ps=2, p_tie=0.1, n_clock=0)
        tune = dict(bins_per_tile_log2=2, gate_block_log2=6, unit_events=16, tile_threads=256)
    P64 = O.power(prob)
    st64, b64 = O.event_trace(prob)
    P, st, b = run(prob, 0, **tune)
    assert np.array_equal(st, st64), "state before group differs"
    assert np.array_equal(b, b64), "bin index differs"
    rel = np.abs(P.astype(np.float64) - P64) / P64
    assert rel.max() <= REL, f"max rel err {rel.max():.3e} at bin {rel.argmax()}"
    P1, _, _ = run(prob, 1)
    assert np.array_equal(P.view(np.uint32), P1.view(np.uint32)), "packed and gate-per-thread paths differ"
