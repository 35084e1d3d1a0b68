"""Parity at the full workload sizes, in the launch configuration bench.py
times (default tuning, validated events), against the FP64 oracle.

* 1M gates, 2e8 events, 50 ps bins: every one of the 2e6 bins within 1e-5
  relative; every event's state and bin bit-exact.
* 5M gates, 1e9 Zipf events, 100 ps bins: every bin within 1e-5 relative.
* 1M gates, 1e8 events (the adjoint workload): the gradient of the smooth
  peak-power loss against the FP64 oracle gradient for every net and gate,
  per element |g - g64| <= 1e-4 * max(|g64|, 1e-3 max|g64|); and against
  central finite differences of the FP64 loss (h = 1e-3 fF on 100 sampled
  nets, 1e-3 relative on the leakage scale of 100 sampled gates) with the same
  bar.
* 64 traces of 1k-20k cycles over one 200k-gate netlist (the batched
  workload as bench.py runs it): the recorded-graph batched waveforms
  bit-identical to per-trace forwards, and the shortest, the longest and two
  other traces within 1e-5 of the oracle.

The oracle runs multi-threaded on the host cores; each case takes seconds.
"""
import sys

import numpy as np
import pytest

import oracle
import synth
from _fd import fd_errors, fd_load, fd_scale, sample_gates, sample_nets
from _problems import to_device_ctx

pytestmark = pytest.mark.gpu
REL = 1e-5


@pytest.fixture(scope="module")
def O():
    return oracle.get()


def _say(msg):
    print(msg, file=sys.stderr, flush=True)


def _rel_ok(P, P64, what):
    rel = np.abs(P.astype(np.float64) - P64) / P64
    assert rel.max() <= REL, f"{what}: max rel err {rel.max():.3e} at bin {int(rel.argmax())}"


def test_full_forward_1m_gates_2e8_events(O):
    prob = synth.make_problem("C2")
    _say("C2 generated")
    ctx, load, lam = to_device_ctx(prob)
    P = ctx.forward(load, lam).cpu().numpy()
    P64 = O.power(prob)
    _rel_ok(P, P64, "C2 bins")
    st, b = ctx.event_trace()
    st, b = st.cpu().numpy(), b.cpu().numpy()
    ctx.close()
    st64, b64 = O.event_trace(prob)
    assert np.array_equal(st, st64), f"C2: {int((st != st64).sum())} event states differ"
    assert np.array_equal(b, b64), f"C2: {int((b != b64).sum())} event bins differ"


def test_full_forward_skew_1e9_events(O):
    prob = synth.make_problem("C3")
    _say("C3 generated")
    ctx, load, lam = to_device_ctx(prob)
    P = ctx.forward(load, lam).cpu().numpy()
    ctx.close()
    _say("C3 forward done")
    _rel_ok(P, O.power(prob), "C3 bins")


def test_full_adjoint_1m_gates_1e8_events(O):
    import torch
    prob = synth.make_problem("C5")
    _say("C5 generated")
    P64 = O.power(prob)
    beta = 1.0 / (0.05 * P64.mean())
    _, gP = oracle.lse_loss_grad(P64, beta)
    gl64, gs64 = O.adjoint(prob, gP)
    ctx, load, lam = to_device_ctx(prob)
    gl, gs = ctx.adjoint(load, lam, torch.from_numpy(np.asarray(gP, np.float32)).to(load.device))
    gl, gs = gl.cpu().numpy().astype(np.float64), gs.cpu().numpy().astype(np.float64)
    ctx.close()
    drv = prob.net.gate_out_net
    for what, a, b in (("d/d load", gl[drv], gl64[drv]), ("d/d leak scale", gs, gs64)):
        r = fd_errors(a, b)
        assert r <= 1.0, f"C5 {what} vs the FP64 gradient: {r:.2f} x the per-element bar"
    rng = np.random.default_rng(5)
    nets = sample_nets(prob, gl64, rng)
    gates = sample_gates(prob, gs64, rng)
    fdl = fd_load(O, prob, P64, beta, nets)
    fds = fd_scale(O, prob, P64, beta, gates)
    _say(f"C5 FD: {len(nets)} nets, {len(gates)} gates")
    rl, rs = fd_errors(gl[nets], fdl), fd_errors(gs[gates], fds)
    assert rl <= 1.0, f"C5 d/d load vs central FD: {rl:.2f} x the bar"
    assert rs <= 1.0, f"C5 d/d leak scale vs central FD: {rs:.2f} x the bar"


def test_full_batched_64_traces(O):
    import torch
    import paper_2609_05960_amd as gtp
    lib, net, traces, bin_ps = synth.make_batch(n_traces=64, cycles=(1000, 20000))
    _say(f"batch generated: {sum(ev.n_events for ev in traces)} events")
    dev = torch.device("cuda", 0)
    ctx = gtp.Context(0)
    ctx.load_library(lib)
    ctx.load_netlist(torch.from_numpy(net.gate_cell).to(dev), torch.from_numpy(net.gate_out_net).to(dev),
                     torch.from_numpy(net.gate_init.view(np.int32)).to(dev), net.n_nets)
    ctx.set_params(vdd=0.8, bin_ps=bin_ps)
    ctx.load_traces([tuple(torch.from_numpy(a).to(dev) for a in (ev.gate_off, ev.t, ev.pin_bit, ev.slew))
                     + (ev.t_end,) for ev in traces], validate=True)
    load = torch.from_numpy(net.net_load).to(dev)
    lam = torch.from_numpy(net.leak_scale).to(dev)
    tot, offs = ctx.batch_bins()
    out = torch.empty(tot, dtype=torch.float32, device=dev)
    ctx.forward_batched(load, lam, out=out, use_graph=True)
    ctx.forward_batched(load, lam, out=out, use_graph=True)  # a replay of the recorded graph
    P = out.cpu().numpy()
    for i in range(len(traces)):
        Pi = ctx.forward_trace(i, load, lam).cpu().numpy()
        assert np.array_equal(P[offs[i]:offs[i + 1]].view(np.uint32), Pi.view(np.uint32)), f"trace {i}"
    ctx.close()
    lens = np.array([ev.n_events for ev in traces])
    for i in sorted({int(lens.argmin()), int(lens.argmax()), 1, 33}):
        prob = synth.Problem(lib, net, traces[i], vdd=0.8, bin_ps=bin_ps, sw_mode=0)
        _rel_ok(P[offs[i]:offs[i + 1]], O.power(prob), f"trace {i}")
