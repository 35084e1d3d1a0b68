"""GPU adjoint against the FP64 oracle gradient, through the C ABI and the
autograd Function.

The oracle's gradient is itself pinned to central finite differences and to
the Euler identity of the leakage scale (tests/test_oracle.py), so agreement
with it carries that check to the GPU path. Bar: per element,
|g_gpu - g_64| <= 1e-4 * max|g_64| (the FP32 values of the kernel summed over
many events; the workload's FD bar is 1e-4).
"""
import numpy as np
import pytest

import oracle
import synth
from _problems import load_golden, to_device_ctx

pytestmark = pytest.mark.gpu
TOL = 1e-4


@pytest.fixture(scope="module")
def O():
    return oracle.get()


def gpu_adjoint(prob, gP, algo=0, **tuning):
    import torch
    ctx, load, lam = to_device_ctx(prob, algo=algo)
    if tuning:
        ctx.set_tuning(algo=algo, **tuning)
    gl, gs = ctx.adjoint(load, lam, torch.from_numpy(np.asarray(gP, np.float32)).to(load.device))
    out = gl.cpu().numpy().astype(np.float64), gs.cpu().numpy().astype(np.float64)
    ctx.close()
    return out


def close(a, b, what):
    """Per-element bar: |a - b| <= TOL * max(|b|, 1e-3 * max|b|)."""
    bar = TOL * np.maximum(np.abs(b), 1e-3 * np.abs(b).max())
    bar = np.maximum(bar, 1e-300)
    r = np.abs(a - b) / bar
    i = int(r.argmax())
    assert r[i] <= 1.0, f"{what}: element {i}: {a[i]:.9e} vs {b[i]:.9e} ({r[i]:.2f} x the bar)"


@pytest.mark.parametrize("algo", [0, 1])
@pytest.mark.parametrize("seed", [1, 2, 3, 4, 5, 6])
def test_random_vs_oracle(O, seed, algo):
    rng = np.random.default_rng(100 + seed)
    prob = synth.make_random_small(seed, n_gates=int(rng.integers(5, 120)), n_cells=int(rng.integers(1, 8)),
                                   i_max=int(rng.integers(1, 5)), n_events=int(rng.integers(100, 30000)),
                                   t_end=int(rng.integers(20000, 400000)), bin_ps=int(rng.choice([7, 50, 100, 333])),
                                   p_tie=float(rng.choice([0.0, 0.3])), n_clock=int(rng.integers(0, 3)))
    gP = rng.normal(size=prob.n_bins)  # signed weights: no cancellation hides a wrong term
    gl64, gs64 = O.adjoint(prob, gP)
    gl, gs = gpu_adjoint(prob, gP, algo=algo)
    drv = prob.net.gate_out_net
    close(gl[drv], gl64[drv], "d/d load")
    close(gs, gs64, "d/d leak scale")
    undriven = np.setdiff1d(np.arange(prob.net.n_nets), drv)
    assert np.all(gl[undriven] == 0.0), "nets without a driver must get a zero gradient"


def test_golden_unit_weights(O):
    prob, fx = load_golden("example_a.json")
    exp = fx["expect"]["sw_mode_0"]["grad_unit_g"]
    gl, gs = gpu_adjoint(prob, np.ones(prob.n_bins))
    assert abs(gl[prob.net.gate_out_net[0]] - exp["load"]) <= 1e-6 * abs(exp["load"]) + 1e-12
    assert abs(gs[0] - exp["leak_scale"]) <= 1e-5 * abs(exp["leak_scale"]) + 1e-12


def test_autograd_peak_loss(O):
    """BinnedPower backward with the smooth peak-power loss equals the oracle
    gradient of the same loss (beta from the forward, held constant)."""
    import torch
    import paper_2609_05960_amd as gtp
    prob = synth.make_random_small(77, n_gates=60, n_cells=6, i_max=4, n_events=20000, t_end=200000, bin_ps=50,
                                   p_tie=0.1, n_clock=1)
    ctx, load, lam = to_device_ctx(prob)
    load = load.clone().requires_grad_(True)
    lam = lam.clone().requires_grad_(True)
    P = gtp.binned_power(ctx, load, lam)
    beta = float(1.0 / (0.05 * P.detach().double().mean().item()))
    loss = gtp.peak_power_loss(P, beta)
    loss.backward()
    P64 = O.power(prob)
    _, gP = oracle.lse_loss_grad(P64, beta)
    gl64, gs64 = O.adjoint(prob, gP)
    drv = prob.net.gate_out_net
    close(load.grad.cpu().numpy().astype(np.float64)[drv], gl64[drv], "autograd d/d load")
    close(lam.grad.cpu().numpy().astype(np.float64), gs64, "autograd d/d leak scale")
    ctx.close()


def test_adjoint_workload_scaled(O):
    """The adjoint workload (1M gates, 100M events, 50 ps bins) at 1/100 scale."""
    prob = synth.make_problem("C5", scale=0.01)
    P64 = O.power(prob)
    beta = 1.0 / (0.05 * P64.mean())
    _, gP = oracle.lse_loss_grad(P64, beta)
    gl64, gs64 = O.adjoint(prob, gP)
    gl, gs = gpu_adjoint(prob, gP)
    drv = prob.net.gate_out_net
    close(gl[drv], gl64[drv], "d/d load")
    close(gs, gs64, "d/d leak scale")


@pytest.mark.parametrize("tl,ue,gb", [(4, 16, 6), (2, 5, 6), (9, 8, 14)])
def test_packed_decompositions(O, tl, ue, gb):
    """Small tiles and gate blocks: many work items, groups shared by two gate
    blocks, regions of one unit; every decomposition matches the oracle."""
    prob = synth.make_random_small(91, n_gates=300, n_cells=3, i_max=4, n_events=40000, t_end=300000, bin_ps=50,
                                   p_tie=0.2, n_clock=2)
    gP = np.random.default_rng(5).normal(size=prob.n_bins)
    gl64, gs64 = O.adjoint(prob, gP)
    gl, gs = gpu_adjoint(prob, gP, algo=0, bins_per_tile_log2=tl, unit_events=ue, gate_block_log2=gb)
    drv = prob.net.gate_out_net
    close(gl[drv], gl64[drv], "d/d load")
    close(gs, gs64, "d/d leak scale")


@pytest.mark.parametrize("algo", [0, 1])
def test_shared_output_net(O, algo):
    """Two gates driving one net: the net's load gradient is the sum of both
    gates' terms (the adjoint's atomic path; unique drivers take plain stores)."""
    prob = synth.make_random_small(23, n_gates=40, n_cells=4, i_max=3, n_events=8000, t_end=100000, bin_ps=50,
                                   p_tie=0.1, n_clock=1)
    out = prob.net.gate_out_net
    out[1] = out[0]
    out[7] = out[0]
    gP = np.random.default_rng(9).normal(size=prob.n_bins)
    gl64, gs64 = O.adjoint(prob, gP)
    gl, gs = gpu_adjoint(prob, gP, algo=algo)
    drv = np.unique(out)
    close(gl[drv], gl64[drv], "d/d load")
    close(gs, gs64, "d/d leak scale")
