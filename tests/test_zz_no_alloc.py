"""The allocation-free forward (gtp_forward_noalloc) through the C ABI.

Two calls in a row on one GPU, the second with a smaller input (fewer gates,
events and bins, so the shared scratch array still holds the first call's
larger contents): each result is bit-identical to gtp_forward on the same
context (the same kernels on other buffers) and within 1e-5 of the FP64 oracle
per bin. The call must not allocate: it is also made while a HIP graph
records it (capture fails on an allocation) and the recorded graph replayed.
"""
import ctypes

import numpy as np
import pytest

import oracle
import synth
from _problems import to_device_ctx

pytestmark = pytest.mark.gpu
REL = 1e-5


def _noalloc(ctx, load, lam, out):
    return ctx.L.gtp_forward_noalloc(ctx.h, ctypes.c_void_p(load.data_ptr()), ctypes.c_void_p(lam.data_ptr()),
                                     ctypes.c_void_p(out.data_ptr()))


def _case(prob):
    import torch
    O = oracle.get()
    ctx, load, lam = to_device_ctx(prob)
    out = torch.full((ctx.n_bins,), -1.0, dtype=torch.float32, device=load.device)
    rc = _noalloc(ctx, load, lam, out)
    assert rc == 4, "before the layout is built the call reports NOT_LOADED"
    ctx.plan_info()                                   # builds the layout (allocating call)
    rc = _noalloc(ctx, load, lam, out)
    assert rc == 0, ctx.L.gtp_last_error(ctx.h)
    ref = ctx.forward(load, lam)
    torch.cuda.synchronize()
    ctx.sync()
    assert torch.equal(out.view(torch.int32), ref.view(torch.int32)), "not bit-identical to gtp_forward"
    P64 = O.power(prob)
    rel = np.abs(out.cpu().numpy().astype(np.float64) - P64) / P64
    assert rel.max() <= REL, f"max rel err {rel.max():.3e}"
    return ctx, load, lam, ref


def test_noalloc_two_calls_second_smaller():
    big = synth.make_problem("C1")
    small = synth.make_random_small(5, n_gates=37, n_cells=5, i_max=4, n_events=4000, t_end=30000, bin_ps=70,
                                    p_tie=0.2, n_clock=1)
    c1, *_ = _case(big)
    c1.close()
    c2, *_ = _case(small)
    c2.close()


def test_noalloc_under_graph_capture():
    import torch
    prob = synth.make_random_small(9, n_gates=50, n_cells=6, i_max=4, n_events=20000, t_end=100000, bin_ps=50,
                                   p_tie=0.1, n_clock=2)
    ctx, load, lam, ref = _case(prob)
    out = torch.empty_like(ref)
    s = torch.cuda.Stream()
    ctx.set_stream(s)
    g = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=s):
        rc = _noalloc(ctx, load, lam, out)
    assert rc == 0, ctx.L.gtp_last_error(ctx.h)
    for k in range(3):
        out.fill_(-1.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out.view(torch.int32), ref.view(torch.int32)), f"replay {k}"
    ctx.set_stream(torch.cuda.current_stream())
    ctx.close()


def test_noalloc_limits():
    """Too many bins for the scratch array: a clear UNSUPPORTED, nothing launched."""
    import torch
    prob = synth.make_random_small(3, n_gates=20, n_events=500, t_end=50_000_000, bin_ps=5)   # 10^7 bins
    ctx, load, lam = to_device_ctx(prob)
    ctx.plan_info()
    out = torch.empty(ctx.n_bins, dtype=torch.float32, device=load.device)
    rc = _noalloc(ctx, load, lam, out)
    assert rc == 8 and b"scratch" in ctx.L.gtp_last_error(ctx.h)
    ctx.close()
