"""Glitch power, the per-gate report, the state index over every pin and the
paper-faithful settings, through the C ABI on the GPU, against the FP64
oracle.

Bars: waveform bins within 1e-5 relative of the oracle and the packed and
one-gate-per-thread paths bit-identical (exact fixed point); per-gate report
components within 1e-6 relative (FP32 per-event energies summed in FP64);
adjoint per element within 1e-4 * max(|g64|, 1e-3 max|g64|); per-event
states bit-exact.
"""
import numpy as np
import pytest

import oracle
import synth
from _problems import all_pin_library, load_golden, to_device_ctx

pytestmark = pytest.mark.gpu
REL = 1e-5


@pytest.fixture(scope="module")
def O():
    return oracle.get()


def _glitchy(seed, allp=0, clk=1000, **kw):
    """A random problem with clock gates (two toggles of pin 0 per cycle) and
    dense random gates, so that many events are glitches."""
    args = dict(n_gates=60, n_cells=6, i_max=3 if allp else 4, n_events=30000, t_end=200000, bin_ps=50, p_tie=0.1,
                n_clock=3)
    args.update(kw)
    prob = synth.make_random_small(seed, **args)
    if allp:
        prob.lib = all_pin_library(prob.lib, seed)
    prob.state_all_pins = allp
    prob.glitch_clk = clk
    return prob


def _forward(prob, algo=0):
    ctx, load, lam = to_device_ctx(prob, algo=algo)
    P = ctx.forward(load, lam)
    ge, summ = ctx.report(load, lam, P)
    st, b = ctx.event_trace()
    out = P.cpu().numpy(), ge.cpu().numpy(), summ, st.cpu().numpy(), b.cpu().numpy()
    ctx.sync()
    ctx.close()
    return out


def _check(prob, O):
    P64 = O.power(prob)
    GE64, tmax64 = O.gate_report(prob)
    st64, b64 = O.event_trace(prob)
    res = [_forward(prob, algo) for algo in (0, 1)]
    for P, ge, summ, st, b in res:
        rel = np.abs(P.astype(np.float64) - P64) / P64
        assert rel.max() <= REL, f"bins: max rel err {rel.max():.3e}"
        np.testing.assert_allclose(ge, GE64, rtol=1e-6, atol=1e-12)
        assert summ["t_max_ps"] == tmax64
        np.testing.assert_allclose([summ["energy_fj"][k] for k in ("leak", "int", "sw", "gl")], GE64.sum(axis=0),
                                   rtol=1e-6)
        assert summ["peak_mw"] == float(P.max())
        assert np.array_equal(st, st64) and np.array_equal(b, b64)
    assert np.array_equal(res[0][0].view(np.uint32), res[1][0].view(np.uint32)), "paths not bit-identical"
    return res[0]


def test_golden_glitch(O):
    """Hand-computed glitch fixture: bins, components and the latest event time."""
    prob, fx = load_golden("example_c.json")
    exp = fx["expect"]
    P, ge, summ, _, _ = _check(prob, O)
    np.testing.assert_allclose(P.astype(np.float64) * prob.bin_ps, exp["bins_fj"], rtol=1e-6)
    c = exp["components_fj"]
    np.testing.assert_allclose(ge[0], [c["leak"], c["int"], c["sw"], c["gl"]], rtol=1e-6)
    assert summ["t_max_ps"] == exp["t_max"]
    np.testing.assert_allclose(summ["avg_mw_tmax"]["gl"], c["gl"] / exp["t_max"], rtol=1e-6)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_glitch_random(O, seed):
    prob = _glitchy(seed)
    _, ge, _, _, _ = _check(prob, O)
    assert ge[:, 3].sum() > 0.05 * ge[:, 1:].sum(), "the case holds many glitch events"


@pytest.mark.parametrize("seed", [4, 5])
def test_all_pin_state(O, seed):
    """State index over every pin (output toggles change the leakage state and
    the table), without and with glitch detection."""
    for clk in (0, 700):
        _check(_glitchy(seed, allp=1, clk=clk), O)


def test_report_without_glitch(O):
    prob = synth.make_problem("C1")
    _, ge, summ, _, _ = _check(prob, O)
    assert np.all(ge[:, 3] == 0.0)


def test_paper_faithful_preset(O):
    """The paper's settings together: per-cycle bins (bin = clock period),
    switching energy C V^2 on output rises, the state over every pin, glitch
    detection per clock cycle, and the averages p = E / t_max."""
    prob = _glitchy(9, allp=1, clk=1000, bin_ps=1000, n_events=20000, t_end=300000)
    prob.sw_mode = 1
    P, ge, summ, _, _ = _check(prob, O)
    GE64, tmax64 = O.gate_report(prob)
    for k, name in enumerate(("leak", "int", "sw", "gl")):
        np.testing.assert_allclose(summ["avg_mw_tmax"][name], GE64[:, k].sum() / tmax64, rtol=1e-6)


@pytest.mark.parametrize("allp,clk", [(0, 1000), (1, 0), (1, 800)])
def test_adjoint_glitch_and_all_pins(O, allp, clk):
    import torch
    prob = _glitchy(21, allp=allp, clk=clk, n_events=20000)
    gP = np.random.default_rng(3).normal(size=prob.n_bins)
    gl64, gs64 = O.adjoint(prob, gP)
    for algo in (0, 1):
        ctx, load, lam = to_device_ctx(prob, algo=algo)
        gl, gs = ctx.adjoint(load, lam, torch.from_numpy(np.asarray(gP, np.float32)).to(load.device))
        gl, gs = gl.cpu().numpy().astype(np.float64), gs.cpu().numpy().astype(np.float64)
        ctx.close()
        drv = prob.net.gate_out_net
        for a, b, what in ((gl[drv], gl64[drv], "load"), (gs, gs64, "scale")):
            bar = 1e-4 * np.maximum(np.abs(b), 1e-3 * np.abs(b).max())
            r = (np.abs(a - b) / bar).max()
            assert r <= 1.0, f"algo {algo} d/d {what}: {r:.2f} x the bar"


def test_batched_glitch(O):
    """Batched traces with glitch detection: bit-identical to per-trace
    forwards, within 1e-5 of the oracle."""
    import torch
    import paper_2609_05960_amd as gtp
    lib, net, traces, bin_ps = synth.make_batch(n_traces=4, cycles=(5, 40), events_per_cycle=600, n_gates=80,
                                                n_cells=5, i_max=4, bin_ps=50, seed=13, p_tie=0.1)
    dev = torch.device("cuda", 0)
    ctx = gtp.Context(0)
    ctx.load_library(lib)
    ctx.load_netlist(torch.from_numpy(net.gate_cell).to(dev), torch.from_numpy(net.gate_out_net).to(dev),
                     torch.from_numpy(net.gate_init.view(np.int32)).to(dev), net.n_nets)
    ctx.set_params(vdd=0.8, bin_ps=bin_ps, glitch_clk_ps=1000)
    ctx.load_traces([tuple(torch.from_numpy(a).to(dev) for a in (ev.gate_off, ev.t, ev.pin_bit, ev.slew))
                     + (ev.t_end,) for ev in traces], validate=True)
    load = torch.from_numpy(net.net_load).to(dev)
    lam = torch.from_numpy(net.leak_scale).to(dev)
    tot, offs = ctx.batch_bins()
    out = ctx.forward_batched(load, lam, use_graph=True)
    P = out.cpu().numpy()
    for i, ev in enumerate(traces):
        Pi = ctx.forward_trace(i, load, lam).cpu().numpy()
        assert np.array_equal(P[offs[i]:offs[i + 1]].view(np.uint32), Pi.view(np.uint32)), f"trace {i}"
        prob = synth.Problem(lib, net, ev, vdd=0.8, bin_ps=bin_ps, glitch_clk=1000)
        rel = np.abs(P[offs[i]:offs[i + 1]].astype(np.float64) - O.power(prob)) / O.power(prob)
        assert rel.max() <= REL, f"trace {i}: {rel.max():.3e}"
    ctx.close()
