"""Central finite differences of the smooth peak-power loss, evaluated with the
FP64 oracle (test infrastructure; the oracle only).

Loss L(P) = (1/beta) log sum_b exp(beta P_b), beta held constant. A change of
one net's load (or one gate's leakage scale) only changes the binned energy of
the gates involved, so L(P + dP) is evaluated from the full FP64 waveform P and
the oracle's energy of those gates alone:

    L(P + dP) - L(P) = (1/beta) log1p( sum_b s_b expm1(beta dP_b) ),
    s = softmax(beta P),

with dP_b = (E_g,b(perturbed) - E_g,b(unperturbed)) / D. Both differences are
formed without cancelling large numbers, so the central difference
(L(+h) - L(-h)) / 2h keeps its precision for gates of any size.

Protocol: 50 nets drawn uniformly over the driven nets plus 50 drawn with
probability proportional to |dL/dC| of the oracle's analytic gradient (so the
checks are not all on negligible nets), h = 1e-3 fF, nets whose load lies
within 2h of a knot of a driving cell's load axis skipped (the bilinear
interpolation has a kink there); the same for the leakage scale of 100 gates
with h = 1e-3 relative. Pass: |g - g_fd| <= tol * max(|g_fd|, 1e-3 max|g_fd|).
"""
import numpy as np


def _dloss(O, prob, s, beta, gates, net_load=None, leak_scale=None, E0=None):
    E = O.forward(prob, gates=gates, net_load=net_load, leak_scale=leak_scale, nthreads=1)
    dP = (E - E0) / float(prob.bin_ps)
    nz = np.nonzero(dP)[0]
    return np.log1p(np.sum(s[nz] * np.expm1(beta * dP[nz]))) / beta


def sample_nets(prob, gl_ref, rng, n_uniform=50, n_weighted=50, h=1e-3):
    """Nets (driven, away from load-axis knots): uniform + proportional to |gl_ref|."""
    net, lib = prob.net, prob.lib
    drv = np.unique(net.gate_out_net)
    C = net.net_load.astype(np.float64)
    ax = lib.load_axis.astype(np.float64).reshape(lib.n_cells, lib.n_load)[net.gate_cell]
    near = np.abs(ax - C[net.gate_out_net][:, None]).min(axis=1) <= 2 * h
    ok = np.ones(net.n_nets, bool)
    ok[net.gate_out_net[near]] = False
    cand = drv[ok[drv]]
    pick = set(rng.choice(cand, size=min(n_uniform, len(cand)), replace=False).tolist())
    w = np.abs(gl_ref[cand])
    if w.sum() > 0:
        pick |= set(rng.choice(cand, size=min(n_weighted, int((w > 0).sum())), replace=False,
                               p=w / w.sum()).tolist())
    return np.array(sorted(pick), np.int64)


def sample_gates(prob, gs_ref, rng, n_uniform=50, n_weighted=50):
    G = prob.net.n_gates
    pick = set(rng.choice(G, size=min(n_uniform, G), replace=False).tolist())
    w = np.abs(gs_ref)
    if w.sum() > 0:
        pick |= set(rng.choice(G, size=min(n_weighted, int((w > 0).sum())), replace=False, p=w / w.sum()).tolist())
    return np.array(sorted(pick), np.int64)


def fd_load(O, prob, P64, beta, nets, h=1e-3):
    """Central FD of the loss w.r.t. the load of each net in `nets`. Loads are
    FP32 inputs, so the step actually taken is the difference of the FP32
    perturbed loads (the quotient uses it, not the nominal 2h)."""
    s = np.exp(beta * (P64 - P64.max()))
    s /= s.sum()
    drivers = {}
    for g, n in enumerate(prob.net.gate_out_net):
        drivers.setdefault(int(n), []).append(g)
    out = np.zeros(len(nets))
    for i, n in enumerate(nets):
        gates = drivers[int(n)]
        E0 = O.forward(prob, gates=gates, nthreads=1)
        c0 = float(prob.net.net_load[n])
        L, steps = [], []
        for sign in (1.0, -1.0):
            load = prob.net.net_load.astype(np.float32).copy()
            load[n] = np.float32(c0 + sign * h)
            steps.append(float(load[n]))
            L.append(_dloss(O, prob, s, beta, gates, net_load=load, E0=E0))
        out[i] = (L[0] - L[1]) / (steps[0] - steps[1])
    return out


def fd_scale(O, prob, P64, beta, gates, h_rel=1e-3):
    """Central FD of the loss w.r.t. the leakage scale of each gate in `gates`
    (FP32 inputs: the quotient uses the step actually taken)."""
    s = np.exp(beta * (P64 - P64.max()))
    s /= s.sum()
    out = np.zeros(len(gates))
    for i, g in enumerate(gates):
        E0 = O.forward(prob, gates=[int(g)], nthreads=1)
        lam0 = float(prob.net.leak_scale[g])
        h = h_rel * max(lam0, 1e-30)
        L, steps = [], []
        for sign in (1.0, -1.0):
            lam = prob.net.leak_scale.astype(np.float32).copy()
            lam[g] = np.float32(lam0 + sign * h)
            steps.append(float(lam[g]))
            L.append(_dloss(O, prob, s, beta, [int(g)], leak_scale=lam, E0=E0))
        out[i] = (L[0] - L[1]) / (steps[0] - steps[1])
    return out


def fd_errors(g, g_fd, tol=1e-4):
    """Largest ratio |g - g_fd| / (tol * max(|g_fd|, 1e-3 max|g_fd|)); <= 1 passes."""
    g = np.asarray(g, np.float64)
    floor = 1e-3 * np.abs(g_fd).max()
    bar = tol * np.maximum(np.abs(g_fd), floor)
    return float((np.abs(g - g_fd) / bar).max())
