"""Error statuses through the C ABI on the GPU.

* Every validation status of gtp_load_events (time outside the window on
  either side, time decreasing, pin above the output pin, pin repeated at one
  time, not a toggle): one planted bad event in a valid trace; the status and
  the reported event equal what the FP64 oracle's own validation finds.
* A failed gtp_load_netlist leaves the ctx without a netlist (later calls
  report NOT_LOADED rather than reading half-loaded arrays).
* A window too large for device memory gives OUT_OF_MEMORY, not a fault.
* A recorded batched graph stays correct after a later gtp_load_events makes
  the library reallocate a scratch buffer the graph used.
"""
import numpy as np
import pytest

import oracle
import synth
from _problems import to_device_ctx

pytestmark = pytest.mark.gpu

STATUS = {"EVENT_ORDER": 5, "EVENT_RANGE": 6, "NOT_TOGGLE": 7}


@pytest.fixture(scope="module")
def O():
    return oracle.get()


def _prob():
    return synth.make_random_small(31, n_gates=30, n_cells=4, i_max=3, n_events=3000, t_end=40000, bin_ps=50,
                                   p_tie=0.2, n_clock=1)


def _gate_with_events(prob, k=3):
    off = prob.ev.gate_off
    return next(g for g in range(prob.net.n_gates) if off[g + 1] - off[g] >= k)


def _plant(prob, kind):
    ev = prob.ev
    t, pb = ev.t.copy(), ev.pin_bit.copy()
    g = _gate_with_events(prob)
    e = int(ev.gate_off[g]) + 1
    I = int(prob.lib.n_inputs[prob.net.gate_cell[g]])
    if kind == "time_high":
        t[e] = ev.t_end
    elif kind == "time_negative":
        t[int(ev.gate_off[g])] = -5
    elif kind == "time_decreasing":
        t[e] = t[e - 1] - 1
    elif kind == "pin_range":
        pb[e] = np.uint8(((I + 1) << 1) | (pb[e] & 1))
    elif kind == "pin_repeat":
        t[e] = t[e - 1]
        pb[e] = pb[e - 1] ^ np.uint8(1)
    elif kind == "not_toggle":
        pb[e] = pb[e] ^ np.uint8(1)
    else:
        raise ValueError(kind)
    return synth.Problem(prob.lib, prob.net, synth.Events(ev.n_events, ev.t_end, ev.gate_off, t, pb, ev.slew),
                         vdd=prob.vdd, bin_ps=prob.bin_ps, sw_mode=prob.sw_mode)


@pytest.mark.parametrize("kind,status", [("time_high", "EVENT_RANGE"), ("time_negative", "EVENT_RANGE"),
                                         ("time_decreasing", "EVENT_ORDER"), ("pin_range", "EVENT_RANGE"),
                                         ("pin_repeat", "EVENT_ORDER"), ("not_toggle", "NOT_TOGGLE")])
def test_validation_status_matches_oracle(O, kind, status):
    import paper_2609_05960_amd as gtp
    bad = _plant(_prob(), kind)
    rc, idx = O.validate(bad)
    assert rc == STATUS[status], f"oracle gives {rc} for {kind}"
    with pytest.raises(gtp.GtpError) as ei:
        to_device_ctx(bad, validate=True)
    assert ei.value.status == status
    assert ei.value.bad_event == idx, f"{kind}: GPU names event {ei.value.bad_event}, oracle {idx}"


def test_valid_trace_passes_validation(O):
    prob = _prob()
    assert O.validate(prob) == (0, -1)
    ctx, load, lam = to_device_ctx(prob, validate=True)
    ctx.close()


def test_failed_netlist_load_leaves_nothing_loaded():
    import torch
    import paper_2609_05960_amd as gtp
    prob = _prob()
    ctx, load, lam = to_device_ctx(prob)
    ctx.forward(load, lam)
    net = prob.net
    dev = load.device
    cell = net.gate_cell.copy()
    cell[3] = prob.lib.n_cells + 5   # no such cell
    with pytest.raises(gtp.GtpError) as ei:
        ctx.load_netlist(torch.from_numpy(cell).to(dev), torch.from_numpy(net.gate_out_net).to(dev),
                         torch.from_numpy(net.gate_init.view(np.int32)).to(dev), net.n_nets)
    assert ei.value.status == "INVALID_ARG"
    with pytest.raises(gtp.GtpError) as ei:
        ctx.forward(load, lam)
    assert ei.value.status == "NOT_LOADED"
    ctx.close()


def test_window_beyond_device_memory_is_out_of_memory():
    import torch
    import paper_2609_05960_amd as gtp
    prob = _prob()
    ctx, load, lam = to_device_ctx(prob)
    ev = prob.ev
    dev = load.device
    tens = [torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in (ev.gate_off, ev.t, ev.pin_bit, ev.slew)]
    ctx.load_events(*tens, t_end=1 << 42, validate=False)   # 2^42 bins of 1 ps: 35 TB of bins
    ctx.set_params(vdd=0.8, bin_ps=1)
    # the binding refuses an output smaller than the bins; the C call checks the
    # bin buffers against the device memory before anything is launched
    with pytest.raises(ValueError):
        ctx.forward(load, lam, out=torch.empty(16, dtype=torch.float32, device=dev))
    out = torch.empty(16, dtype=torch.float32, device=dev)
    rc = ctx.L.gtp_forward(ctx.h, load.data_ptr(), lam.data_ptr(), out.data_ptr())
    assert gtp.STATUS[rc] == "OUT_OF_MEMORY", ctx.L.gtp_last_error(ctx.h)
    ctx.close()


def test_graph_survives_scratch_reallocation(O):
    """Batched graph recorded, then a long single trace is loaded (its plan
    scan needs a larger scratch than the batch's), then the graph is used again
    with the same pointers: it must be re-recorded, not replayed on freed
    memory."""
    import torch
    import paper_2609_05960_amd as gtp
    lib, net, traces, bin_ps = synth.make_batch(n_traces=3, cycles=(3, 10), events_per_cycle=200, n_gates=60,
                                                n_cells=4, i_max=3, bin_ps=50, seed=11)
    dev = torch.device("cuda", 0)
    ctx = gtp.Context(0)
    ctx.load_library(lib)
    ctx.load_netlist(torch.from_numpy(net.gate_cell).to(dev), torch.from_numpy(net.gate_out_net).to(dev),
                     torch.from_numpy(net.gate_init.view(np.int32)).to(dev), net.n_nets)
    ctx.set_params(vdd=0.8, bin_ps=bin_ps)
    ctx.load_traces([tuple(torch.from_numpy(a).to(dev) for a in (ev.gate_off, ev.t, ev.pin_bit, ev.slew))
                     + (ev.t_end,) for ev in traces])
    load = torch.from_numpy(net.net_load).to(dev)
    lam = torch.from_numpy(net.leak_scale).to(dev)
    tot, offs = ctx.batch_bins()
    out = torch.empty(tot, dtype=torch.float32, device=dev)
    ctx.forward_batched(load, lam, out=out, use_graph=True)
    ref = out.clone()
    # a long trace over the same netlist: 2^22 events, far more scan tiles than the batch's bins
    long = synth.make_events(99, lib, net, np.full(net.n_gates, (1 << 22) // net.n_gates, np.int64),
                             np.zeros(net.n_gates, np.uint8), t_end=(1 << 22), t_clk=1000)
    lt = [torch.from_numpy(a).to(dev) for a in (long.gate_off, long.t, long.pin_bit, long.slew)]
    ctx.load_events(*lt, t_end=long.t_end, validate=False)
    ctx.forward(load, lam)
    out.fill_(-1.0)
    ctx.forward_batched(load, lam, out=out, use_graph=True)
    torch.cuda.synchronize()
    assert torch.equal(out.view(torch.int32), ref.view(torch.int32))
    ctx.close()
