"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Nothing here compares the oracle with itself: every expected value comes from
a hand-worked fixture, a closed form, a brute-force evaluation written in a
different formulation (per-picosecond leakage integration, toggle-parity
states, a library interpolator), or an identity the method must satisfy.
``test_planted_mistakes_are_caught`` rebuilds the oracle with deliberate
mistakes and checks that at least one pin fails for each.
"""
import itertools
import json
import os

import numpy as np
import pytest
from scipy.interpolate import RegularGridInterpolator

import oracle
import synth
from _problems import GOLDEN, all_pin_library, build_problem, load_golden

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")


@pytest.fixture(scope="module")
def O():
    oracle.build()
    return oracle.get()


# ---------------------------------------------------------------------------
# pins, each a function of an Oracle so the planted-mistake test can reuse them
# ---------------------------------------------------------------------------

def pin_golden_a(O):
    """Hand-computed one-input waveform (fixture example_a)."""
    for mode, key in ((0, "sw_mode_0"), (1, "sw_mode_1")):
        prob, fx = load_golden("example_a.json", sw_mode=mode)
        exp = fx["expect"][key]
        E = O.forward(prob)
        np.testing.assert_allclose(E, exp["bins_fj"], rtol=1e-12, atol=1e-15)
        assert abs(E.sum() - exp["total_fj"]) < 1e-12
    prob, fx = load_golden("example_a.json")
    exp = fx["expect"]["sw_mode_0"]
    st, b = O.event_trace(prob)
    assert st.tolist() == exp["state_before"] and b.tolist() == exp["bin"]
    for mode in (0, 1):
        gl, gs = O.adjoint(prob, np.ones(prob.n_bins), leak_mode=mode)
        assert abs(gl[prob.net.gate_out_net[0]] - exp["grad_unit_g"]["load"]) < 1e-14
        assert abs(gs[0] - exp["grad_unit_g"]["leak_scale"]) < 1e-15


def pin_golden_b(O):
    """Hand-computed two-input waveform with a simultaneous pair (example_b)."""
    prob, fx = load_golden("example_b.json")
    exp = fx["expect"]["sw_mode_0"]
    E, tot = O.forward(prob, return_totals=True)
    np.testing.assert_allclose(E, exp["bins_fj"], rtol=1e-12, atol=1e-15)
    c = exp["components_fj"]
    np.testing.assert_allclose(tot[:3], [c["int"], c["sw"], c["leak"]], rtol=1e-12)
    assert tot[3] == 0.0
    st, b = O.event_trace(prob)
    assert st.tolist() == exp["state_before"] and b.tolist() == exp["bin"]
    gl, gs = O.adjoint(prob, np.ones(prob.n_bins))
    assert abs(gl[prob.net.gate_out_net[0]] - exp["grad_unit_g"]["load"]) < 1e-13
    assert abs(gs[0] - exp["grad_unit_g"]["leak_scale"]) < 1e-15


def pin_golden_c(O):
    """Hand-computed glitch waveform and per-gate components (fixture example_c)."""
    prob, fx = load_golden("example_c.json")
    exp = fx["expect"]
    E, tot = O.forward(prob, return_totals=True)
    np.testing.assert_allclose(E, exp["bins_fj"], rtol=1e-12, atol=1e-15)
    c = exp["components_fj"]
    np.testing.assert_allclose(tot, [c["int"], c["sw"], c["leak"], c["gl"]], rtol=1e-12)
    assert abs(E.sum() - exp["total_fj"]) < 1e-12
    GE, tmax = O.gate_report(prob)
    np.testing.assert_allclose(GE[0], [c["leak"], c["int"], c["sw"], c["gl"]], rtol=1e-12)
    assert tmax == exp["t_max"]
    prob.glitch_clk = 0
    np.testing.assert_allclose(O.forward(prob), exp["no_glitch_bins_fj"], rtol=1e-12, atol=1e-15)


def pin_bin_index(O):
    """bin = floor(t / D), half-open bins: exhaustive on [0, 10D] plus edges."""
    D = 100
    ts = list(range(0, 10 * D)) + [D * 10 - 1]
    events = []
    val = 0
    for t in ts[: 10 * D]:
        val ^= 1
        events.append((0, t, 0, val, 50.0))
    cell = dict(n_inputs=1, slew_axis=[10.0, 100.0], load_axis=[1.0, 10.0], leak=[1.0, 1.0],
                table_fn=lambda s, d: np.ones((2, 2)))
    prob = build_problem([cell], [dict(cell=0, init=[0, 0], load=1.0)], events, t_end=10 * D, bin_ps=D)
    st, b = O.event_trace(prob)
    assert b.tolist() == [t // D for t in ts[: 10 * D]]
    # state before alternates 0,1,0,... (one input pin toggling)
    assert st.tolist() == [k % 2 for k in range(10 * D)]


def pin_interp(O):
    """Knots exact; bilinear tables reproduced everywhere (extrapolation too);
    a non-bilinear table matches a library linear interpolator inside the grid."""
    sa = [5.0, 20.0, 60.0, 200.0, 500.0]
    la = [0.5, 2.0, 7.0, 20.0, 50.0]
    a0, a1, a2, a3 = 0.3, 0.011, 0.07, 0.0009

    def fbil(s, C):
        return a0 + a1 * s + a2 * C + a3 * s * C

    S, Cg = np.meshgrid(sa, la, indexing="ij")
    Tb = fbil(S, Cg)
    Tn = 0.1 + np.sqrt(S * Cg) / 10.0 + (S / 100.0) ** 2
    cell = dict(n_inputs=1, slew_axis=sa, load_axis=la, leak=[1.0, 2.0],
                table_fn=lambda s, d: Tb if (s, d) == (0, 0) else Tn)
    prob = build_problem([cell], [dict(cell=0, init=[0, 0], load=1.0)], [], t_end=100, bin_ps=10)
    Tn32 = Tn.astype(np.float32).astype(np.float64)
    Tb32 = Tb.astype(np.float32).astype(np.float64)
    for i, s in enumerate(sa):
        for j, C in enumerate(la):
            assert O.bilerp(prob, 0, 1, s, C) == Tn32[i, j]
    rng = np.random.default_rng(0)
    # exact bilinear reproduction: use the float32-rounded table as the target
    rgi_b = RegularGridInterpolator((np.array(sa, np.float32).astype(float), np.array(la, np.float32).astype(float)),
                                    Tb32, method="linear", bounds_error=False, fill_value=None)
    for s, C in zip(rng.uniform(0.5, 900.0, 300), rng.uniform(0.05, 90.0, 300)):
        got = O.bilerp(prob, 0, 0, s, C)
        assert abs(got - rgi_b([[s, C]])[0]) < 1e-9 * max(1.0, abs(got))
        assert abs(got - fbil(s, C)) < 1e-5 * max(1.0, abs(fbil(s, C)))  # float32 table rounding only
    rgi = RegularGridInterpolator((np.array(sa, np.float32).astype(float), np.array(la, np.float32).astype(float)),
                                  Tn32, method="linear", bounds_error=False, fill_value=None)
    for s, C in zip(rng.uniform(1.0, 800.0, 300), rng.uniform(0.1, 80.0, 300)):
        assert abs(O.bilerp(prob, 0, 1, s, C) - rgi([[s, C]])[0]) < 1e-12 * 100
    # on a knot line the value is the 1-D lerp along the other axis
    for C in rng.uniform(0.5, 50.0, 50):
        j = max(0, min(len(la) - 2, int(np.searchsorted(la, C, side="right")) - 1))
        w = (C - la[j]) / (la[j + 1] - la[j])
        assert abs(O.bilerp(prob, 0, 1, 60.0, C) - ((1 - w) * Tn32[2, j] + w * Tn32[2, j + 1])) < 1e-12


def pin_switching(O):
    """0.5 * 10 fF * 0.8^2 = 3.2 fJ per output toggle; C*V^2 on rise in sw_mode 1."""
    cell = dict(n_inputs=1, slew_axis=[10.0, 100.0], load_axis=[1.0, 100.0], leak=[0.0, 0.0],
                table_fn=lambda s, d: np.zeros((2, 2)))
    ev = [(0, 100, 1, 1, 50.0), (0, 300, 1, 0, 50.0)]
    for mode, expect in ((0, [3.2, 3.2]), (1, [6.4, 0.0])):
        prob = build_problem([cell], [dict(cell=0, init=[0, 0], load=10.0)], ev, 400, 100, sw_mode=mode)
        E = O.forward(prob)
        assert abs(E[1] - expect[0]) < 1e-12 and abs(E[3] - expect[1]) < 1e-12
        assert abs(E[0]) < 1e-15 and abs(E[2]) < 1e-15


def pin_leakage_closed_form(O):
    """Event-free trace: P_b = 1e-6 * sum_g lambda_g * leak[s0_g] mW in every bin
    (a partial last bin carries its share over the full bin width)."""
    lib = synth.make_library(11, 5, 4)
    net = synth.make_netlist(11, lib, 37)
    net.leak_scale = np.random.default_rng(3).uniform(0.2, 3.0, 37).astype(np.float32)
    ev = synth.Events(0, 1050, np.zeros(38, np.int64), np.zeros(0, np.int64), np.zeros(0, np.uint8),
                      np.zeros(0, np.float32))
    prob = synth.Problem(lib, net, ev, vdd=0.8, bin_ps=100)
    rate = 0.0
    for g in range(37):
        c = net.gate_cell[g]
        I = lib.n_inputs[c]
        s0 = int(net.gate_init[g]) & ((1 << I) - 1)
        rate += float(net.leak_scale[g]) * float(lib.leak[lib.leak_base[c] + s0])
    for mode in (0, 1):
        P = O.power(prob, leak_mode=mode)
        np.testing.assert_allclose(P[:10], 1e-6 * rate, rtol=1e-13)
        assert abs(P[10] - 1e-6 * rate * 50 / 100) < 1e-13 * rate


def _match(care, value, s):
    """First pattern whose named pins all carry the values it gives, checked
    pin by pin (-1: none)."""
    for k in range(len(care)):
        if all(((s >> p) & 1) == ((int(value[k]) >> p) & 1) for p in range(32) if (int(care[k]) >> p) & 1):
            return k
    return -1


def _table_id(lib, c, s, d):
    if lib.n_tpat is not None and lib.n_tpat[c] > 0:
        b, n = int(lib.tpat_base[c]), int(lib.n_tpat[c])
        k = _match(lib.tpat_care[b:b + n], lib.tpat_value[b:b + n], s)
        return int(lib.tpat_table[2 * (b + k) + d])
    return int(lib.state_to_table[lib.map_base[c] + 2 * s + d])


def _leak_nw(lib, c, s):
    if lib.n_tpat is not None and lib.n_tpat[c] > 0:
        b, n = int(lib.lpat_base[c]), int(lib.n_lpat[c])
        return float(lib.lpat_leak[b + _match(lib.lpat_care[b:b + n], lib.lpat_value[b:b + n], s)])
    return float(lib.leak[lib.leak_base[c] + s])


def _bruteforce(prob):
    """Plain-definition waveform and per-gate energies: dynamic energy of every
    event in its bin, and leakage integrated picosecond by picosecond at the
    state given by toggle parity (init bit XOR number of events on the pin at
    or before t). Interpolation by a library linear interpolator on the
    float32 tables. Glitches (prob.glitch_clk > 0): an event is a glitch when
    its pin's previous event lies in the same clock cycle; its dynamic energy
    is scaled by min(1, (2 * gap / (sum of the two slews))^2) and counted as
    glitch energy. Returns (bins [n_bins], per-gate [G, 4] = leak, int, sw, gl)."""
    lib, net, ev = prob.lib, prob.net, prob.ev
    nb = prob.n_bins
    E = np.zeros(nb)
    GE = np.zeros((net.n_gates, 4))
    ns, nl = lib.n_slew, lib.n_load
    allp = int(getattr(prob, "state_all_pins", 0))
    T = int(getattr(prob, "glitch_clk", 0))
    for g in range(net.n_gates):
        c = int(net.gate_cell[g])
        I = int(lib.n_inputs[c])
        C = float(net.net_load[net.gate_out_net[g]])
        lam = float(net.leak_scale[g])
        o0, o1 = int(ev.gate_off[g]), int(ev.gate_off[g + 1])
        ts = ev.t[o0:o1]
        pins = ev.pin_bit[o0:o1] >> 1
        vals = ev.pin_bit[o0:o1] & 1
        sl = ev.slew[o0:o1].astype(np.float64)
        init = int(net.gate_init[g])

        def state_at(t, strict):
            s = 0
            for p in range(I + allp):
                m = (ts < t) if strict else (ts <= t)
                n = int(np.count_nonzero(m & (pins == p)))
                s |= (((init >> p) & 1) ^ (n & 1)) << p
            return s

        sa = lib.slew_axis[c * ns:(c + 1) * ns].astype(float)
        la = lib.load_axis[c * nl:(c + 1) * nl].astype(float)
        for q in range(o1 - o0):
            t = int(ts[q])
            s = state_at(t, strict=True)  # state before the event's timestamp
            k = _table_id(lib, c, s, int(vals[q]))
            Tab = lib.tables[(lib.table_base[c] + k) * ns * nl:(lib.table_base[c] + k + 1) * ns * nl]
            rgi = RegularGridInterpolator((sa, la), Tab.reshape(ns, nl).astype(float), method="linear",
                                          bounds_error=False, fill_value=None)
            ei = rgi([[float(ev.slew[o0 + q]), C]])[0]
            es = 0.0
            if pins[q] == I:
                es = (0.5 * C * prob.vdd ** 2) if prob.sw_mode == 0 else (C * prob.vdd ** 2 * vals[q])
            r = -1.0
            if T > 0:
                prev = [j for j in range(q) if pins[j] == pins[q]]
                if prev and ts[prev[-1]] // T == t // T:
                    j = prev[-1]
                    r = min(1.0, (2.0 * (t - int(ts[j])) / (sl[q] + sl[j])) ** 2)
            if r > 0:
                E[t // prob.bin_ps] += r * (ei + es)
                GE[g, 3] += r * (ei + es)
            else:
                E[t // prob.bin_ps] += ei + es
                GE[g, 1] += ei
                GE[g, 2] += es
        leak_of = {}
        for t in range(ev.t_end):
            s = state_at(t, strict=False)
            if s not in leak_of:
                leak_of[s] = _leak_nw(lib, c, s)
            e = lam * leak_of[s] * 1e-6
            E[t // prob.bin_ps] += e
            GE[g, 0] += e
    return E, GE


def _bruteforce_bins(prob):
    return _bruteforce(prob)[0]


def pin_bruteforce_random(O):
    """Random tiny problems (ties included) against the brute-force definition:
    the waveform and the per-gate report, with and without glitch detection,
    state over the inputs or over every pin."""
    for seed in (1, 2, 3):
        for allp, T in ((0, 0), (0, 100), (1, 0), (1, 150)):
            prob = synth.make_random_small(seed, n_gates=6, n_cells=3, i_max=3, n_events=60, t_end=700, bin_ps=70,
                                           p_tie=0.3)
            if allp:
                prob.lib = all_pin_library(prob.lib, seed)
            prob.state_all_pins, prob.glitch_clk = allp, T
            Ebf, GEbf = _bruteforce(prob)
            for mode in (0, 1):
                E = O.forward(prob, leak_mode=mode)
                np.testing.assert_allclose(E, Ebf, rtol=1e-9, atol=1e-12)
            GE, tmax = O.gate_report(prob)
            np.testing.assert_allclose(GE, GEbf, rtol=1e-9, atol=1e-12)
            assert tmax == int(prob.ev.t.max())
            if T:
                assert GEbf[:, 3].sum() > 0, "the case holds glitches"


def pin_when_golden(O):
    """Hand-computed first-match items of the state-pattern fixture."""
    with open(os.path.join(GOLDEN, "when_patterns.json")) as f:
        fx = json.load(f)
    for case in (fx, fx["partial"]):
        got = [O.pattern_scan(case["care"], case["value"], st) for st in range(1 << fx["n_pins"])]
        assert got == case["expect_first_match"], got


def pin_patterns_random(O):
    """Random tiny problems whose cells are given by state patterns (two cells
    converted, two wide cells of 9 and 11 inputs) against the brute-force
    definition with the pin-by-pin pattern match; state over the inputs and
    over every pin, with and without glitch detection."""
    for seed, allp, T in ((11, 0, 0), (12, 1, 0), (13, 0, 120), (14, 1, 90)):
        prob = synth.make_random_small(seed, n_gates=6, n_cells=3, i_max=3, n_events=70, t_end=600, bin_ps=60,
                                       p_tie=0.3)
        if allp:
            prob.lib = all_pin_library(prob.lib, seed)
        lib = synth.add_pattern_cells(prob.lib, seed, wide_inputs=(9, 11), convert=(0, 2), all_pins=allp,
                                      n_pat=(1, 5), max_care=2)
        net = synth.make_netlist(seed, lib, 8)
        counts, clk = synth.make_counts(seed, 8, 0, 0, "lognormal", 1.0, 1.0, 90, 600)
        prob = synth.Problem(lib, net, synth.make_events(seed, lib, net, counts, clk, 600, 1000, p_tie=0.3),
                             vdd=0.8, bin_ps=60, state_all_pins=allp, glitch_clk=T)
        assert set(net.gate_cell.tolist()) & {0, 2, 3, 4}, "patterned cells are used"
        Ebf, GEbf = _bruteforce(prob)
        np.testing.assert_allclose(O.forward(prob), Ebf, rtol=1e-9, atol=1e-12)
        GE, _ = O.gate_report(prob)
        np.testing.assert_allclose(GE, GEbf, rtol=1e-9, atol=1e-12)


def pin_state_enumeration(O):
    """Exhaustive: I = 1..4, every init state, every sequence of up to 4 events
    over the I+1 pins at times drawn from {10, 20} (so ties occur), in order.
    state_before must equal the toggle-parity state before the timestamp."""
    n_checked = 0
    for I in range(1, 5):
        cell = dict(n_inputs=I, slew_axis=[10.0, 100.0], load_axis=[1.0, 10.0], leak=[1.0] * (1 << I),
                    table_fn=lambda s, d: np.ones((2, 2)))
        npins = I + 1
        max_len = 4 if I <= 2 else 3
        for init in range(1 << npins):
            for L in range(1, max_len + 1):
                for pins in itertools.product(range(npins), repeat=L):
                    for split in range(L + 1):  # first `split` events at t=10, rest at t=20
                        g1, g2 = pins[:split], pins[split:]
                        if len(set(g1)) != len(g1) or len(set(g2)) != len(g2):
                            continue  # a pin may toggle once per timestamp
                        val = init
                        events = []
                        for q, p in enumerate(pins):
                            val ^= 1 << p
                            events.append((0, 10 if q < split else 20, p, (val >> p) & 1, 50.0))
                        prob = build_problem([cell], [dict(cell=0, init_bits=init, load=1.0)], events, 40, 10)
                        st, b = O.event_trace(prob)
                        for q in range(L):
                            tq = 10 if q < split else 20
                            exp = 0
                            for p in range(I):
                                n = sum(1 for r in range(L) if pins[r] == p and (10 if r < split else 20) < tq)
                                exp |= (((init >> p) & 1) ^ (n & 1)) << p
                            assert st[q] == exp, (I, init, pins, split, q)
                            assert b[q] == tq // 10
                        n_checked += 1
    assert n_checked > 1000


def pin_energy_invariant(O):
    """sum_b E_b = E_int + E_sw + E_leak, the totals accumulated without binning."""
    prob = synth.make_random_small(7, n_gates=40, n_cells=5, i_max=4, n_events=3000, t_end=20000, bin_ps=50,
                                   p_tie=0.1, n_clock=2)
    for mode in (0, 1):
        E, tot = O.forward(prob, leak_mode=mode, return_totals=True)
        assert abs(E.sum() - tot.sum()) < 1e-11 * tot.sum()


def pin_adjoint_fd(O):
    """Gradients of a smooth loss against central finite differences of the FP64 forward."""
    prob = synth.make_random_small(5, n_gates=12, n_cells=3, i_max=3, n_events=300, t_end=3000, bin_ps=100,
                                   p_tie=0.1)
    P0 = O.power(prob)
    beta = 1.0 / (0.05 * P0.mean())

    def loss(load, scale):
        P = O.power(prob, net_load=load, leak_scale=scale)
        return oracle.lse_loss_grad(P, beta)[0]

    _, gP = oracle.lse_loss_grad(P0, beta)
    gl, gs = O.adjoint(prob, gP)
    load = prob.net.net_load.astype(np.float64)
    scale = prob.net.leak_scale.astype(np.float64)
    # FD needs float64 inputs: the marshalling casts to float32, so step by a
    # representable amount and divide by the realized step
    for g in range(prob.net.n_gates):
        n = int(prob.net.gate_out_net[g])
        h = 1e-2
        lp, lm = load.copy(), load.copy()
        lp[n] = np.float32(load[n] + h); lm[n] = np.float32(load[n] - h)
        fd = (loss(lp, scale) - loss(lm, scale)) / (float(lp[n]) - float(lm[n]))
        assert abs(gl[n] - fd) <= 1e-4 * max(abs(fd), 1e-6) + 1e-9, (g, gl[n], fd)
        sp, sm = scale.copy(), scale.copy()
        sp[g] = np.float32(scale[g] * 1.01); sm[g] = np.float32(scale[g] * 0.99)
        fd = (loss(load, sp) - loss(load, sm)) / (float(sp[g]) - float(sm[g]))
        assert abs(gs[g] - fd) <= 1e-6 * max(abs(fd), 1e-9) + 1e-12, (g, gs[g], fd)


def pin_euler_identity(O):
    """Leakage is homogeneous of degree 1 in lambda: sum_g lambda_g dL/dlambda_g = sum_b g_b P_b^leak."""
    prob = synth.make_random_small(9, n_gates=30, n_cells=4, i_max=4, n_events=2000, t_end=8000, bin_ps=40)
    rng = np.random.default_rng(1)
    gP = rng.normal(size=prob.n_bins)
    _, gs = O.adjoint(prob, gP)
    P = O.power(prob)
    P_dyn = O.power(prob, leak_scale=np.zeros(prob.net.n_gates, np.float32))
    lhs = float(np.dot(prob.net.leak_scale.astype(np.float64), gs))
    rhs = float(np.dot(gP, P - P_dyn))
    assert abs(lhs - rhs) < 1e-9 * max(1.0, abs(rhs))


PINS = [pin_golden_a, pin_golden_b, pin_golden_c, pin_bin_index, pin_interp, pin_switching, pin_leakage_closed_form,
        pin_bruteforce_random, pin_state_enumeration, pin_energy_invariant, pin_adjoint_fd, pin_euler_identity,
        pin_when_golden, pin_patterns_random]


@pytest.mark.parametrize("pin", PINS, ids=[p.__name__ for p in PINS])
def test_pin(O, pin):
    pin(O)


def test_leak_modes_agree(O):
    """The bin-by-bin and difference-array leakage accumulations give the same bins."""
    prob = synth.make_problem("C1", scale=0.1)
    E0 = O.forward(prob, leak_mode=0)
    E1 = O.forward(prob, leak_mode=1)
    np.testing.assert_allclose(E0, E1, rtol=1e-12, atol=1e-15)
    g = np.random.default_rng(0).normal(size=prob.n_bins)
    a0 = O.adjoint(prob, g, leak_mode=0)
    a1 = O.adjoint(prob, g, leak_mode=1)
    for x, y in zip(a0, a1):
        np.testing.assert_allclose(x, y, rtol=1e-10, atol=1e-14)


def test_gate_permutation_and_window(O):
    """Gate order does not matter; a bin window equals the slice of the full waveform."""
    prob = synth.make_random_small(4, n_gates=50, n_events=4000, t_end=10000, bin_ps=50)
    E = O.forward(prob)
    perm = np.random.default_rng(2).permutation(prob.net.n_gates)
    np.testing.assert_allclose(O.forward(prob, gates=perm), E, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(O.forward(prob, b0=30, b1=120), E[30:120], rtol=1e-12, atol=1e-15)
    half = O.forward(prob, gates=np.arange(25)) + O.forward(prob, gates=np.arange(25, 50))
    np.testing.assert_allclose(half, E, rtol=1e-12, atol=1e-15)


def test_lambda_linearity(O):
    prob = synth.make_random_small(6, n_gates=20, n_events=800)
    lam = prob.net.leak_scale.astype(np.float32)
    E1 = O.forward(prob, leak_scale=lam)
    E0 = O.forward(prob, leak_scale=np.zeros_like(lam))
    E2 = O.forward(prob, leak_scale=2 * lam)
    np.testing.assert_allclose(E2 - E0, 2 * (E1 - E0), rtol=1e-10, atol=1e-15)


def test_error_statuses(O):
    cell = dict(n_inputs=2, slew_axis=[10.0, 100.0], load_axis=[1.0, 10.0], leak=[1.0] * 4,
                table_fn=lambda s, d: np.ones((2, 2)))
    g = [dict(cell=0, init=[0, 0, 0], load=1.0)]
    cases = {
        oracle.ERR_NOT_TOGGLE: [(0, 10, 0, 0, 5.0)],
        oracle.ERR_EVENT_RANGE: [(0, 10, 3, 1, 5.0)],
        oracle.ERR_EVENT_ORDER: [(0, 10, 0, 1, 5.0), (0, 10, 0, 0, 5.0)],
    }
    for code, ev in cases.items():
        prob = build_problem([cell], g, ev, 100, 10)
        rc, bad = O.validate(prob)
        assert rc == code
        with pytest.raises(oracle.OracleError):
            O.forward(prob)
    prob = build_problem([cell], g, [(0, 100, 0, 1, 5.0)], 100, 10)
    assert O.validate(prob)[0] == oracle.ERR_EVENT_RANGE


def test_generator_properties():
    """Generator: exact totals, strictly ordered times per gate (ties only as
    groups of distinct pins), alternating values per pin, determinism."""
    prob = synth.make_problem("C1")
    ev, net, lib = prob.ev, prob.net, prob.lib
    assert ev.n_events == 100_000 and ev.gate_off[-1] == 100_000
    counts = np.diff(ev.gate_off)
    assert (counts == 1999).sum() >= 10
    assert ev.t.min() >= 0 and ev.t.max() < ev.t_end
    assert np.all(ev.slew >= 5.0) and np.all(ev.slew <= 500.0)
    prob2 = synth.make_problem("C1")
    assert np.array_equal(prob2.ev.t, ev.t) and np.array_equal(prob2.ev.slew, ev.slew)
    assert O_free_validate(prob)
    tied = synth.make_random_small(3, n_events=2000, p_tie=0.3)
    assert O_free_validate(tied)
    assert np.any(np.diff(tied.ev.t) == 0)


def O_free_validate(prob):
    """Order / alternation check written with numpy only."""
    ev, net, lib = prob.ev, prob.net, prob.lib
    for g in range(net.n_gates):
        o0, o1 = ev.gate_off[g], ev.gate_off[g + 1]
        t = ev.t[o0:o1]
        if np.any(np.diff(t) < 0):
            return False
        I = lib.n_inputs[net.gate_cell[g]]
        v = int(net.gate_init[g])
        last_t = {}
        for q in range(o1 - o0):
            p, b = int(ev.pin_bit[o0 + q]) >> 1, int(ev.pin_bit[o0 + q]) & 1
            if p > I or ((v >> p) & 1) == b or last_t.get(p) == t[q]:
                return False
            v ^= 1 << p
            last_t[p] = t[q]
    return True


PLANTS = {1: "intermediate state in a group", 2: "transposed table", 3: "switching 2x", 4: "leak after-state",
          5: "rounded bin", 6: "tail leakage dropped", 7: "wrong direction table", 9: "switching term dropped in grad",
          10: "partial bins dropped in grad", 11: "glitch ratio without the factor 2",
          12: "glitch energy unscaled in the waveform", 13: "output left out of an all-pin state",
          14: "pattern value bits outside its care pins compared"}


@pytest.mark.parametrize("plant", sorted(PLANTS), ids=[PLANTS[k] for k in sorted(PLANTS)])
def test_planted_mistakes_are_caught(tmp_path, plant):
    so = oracle.build(force=True, plant=plant, out=str(tmp_path / f"liborc_plant{plant}.so"))
    bad = oracle.Oracle(so_path=so)
    failed = []
    for pin in PINS:
        try:
            pin(bad)
        except (AssertionError, oracle.OracleError):
            failed.append(pin.__name__)
    assert failed, f"planted mistake '{PLANTS[plant]}' passed every pin"


def test_adjoint_fd_protocol_scaled_workload(O):
    """The oracle's analytic gradient of the smooth peak-power loss against
    central finite differences of its own FP64 forward, with the adjoint
    workload's protocol (100 nets: 50 uniform, 50 by |gradient|, h = 1e-3 fF,
    knots skipped; 100 leakage scales, h = 1e-3 relative) on the 1M-gate,
    1e8-event recipe at 1/100 scale. Bar: 1e-6 x max(|g_fd|, 1e-3 max|g_fd|)
    (FP64 on both sides; the GPU's bar is 1e-4)."""
    from _fd import fd_errors, fd_load, fd_scale, sample_gates, sample_nets
    prob = synth.make_problem("C5", scale=0.01)
    P64 = O.power(prob)
    beta = 1.0 / (0.05 * P64.mean())
    _, gP = oracle.lse_loss_grad(P64, beta)
    gl, gs = O.adjoint(prob, gP)
    rng = np.random.default_rng(7)
    nets = sample_nets(prob, gl, rng)
    gates = sample_gates(prob, gs, rng)
    assert len(nets) >= 80 and len(gates) >= 80
    assert fd_errors(gl[nets], fd_load(O, prob, P64, beta, nets), tol=1e-6) <= 1.0
    assert fd_errors(gs[gates], fd_scale(O, prob, P64, beta, gates), tol=1e-6) <= 1.0
