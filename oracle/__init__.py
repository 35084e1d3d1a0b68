"""FP64 reference evaluator (the oracle) — TEST INFRASTRUCTURE ONLY.

Only tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` import this package. The product library never does, and the
two share no code. See oracle.c for what it computes and the paper passages
each step follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")

OK, ERR_INVALID_ARG, ERR_EVENT_ORDER, ERR_EVENT_RANGE, ERR_NOT_TOGGLE = 0, 1, 5, 6, 7
STATUS_NAMES = {0: "OK", 1: "INVALID_ARG", 5: "EVENT_ORDER", 6: "EVENT_RANGE", 7: "NOT_TOGGLE"}


class OracleError(RuntimeError):
    def __init__(self, code: int, bad_event: int = -1):
        super().__init__(f"oracle status {STATUS_NAMES.get(code, code)} at event {bad_event}")
        self.code = code
        self.name = STATUS_NAMES.get(code, str(code))
        self.bad_event = bad_event


class _Problem(ctypes.Structure):
    _fields_ = [
        ("n_cells", ctypes.c_int32), ("n_slew", ctypes.c_int32), ("n_load", ctypes.c_int32),
        ("n_inputs", ctypes.c_void_p), ("slew_axis", ctypes.c_void_p), ("load_axis", ctypes.c_void_p),
        ("map_base", ctypes.c_void_p), ("state_to_table", ctypes.c_void_p), ("table_base", ctypes.c_void_p),
        ("tables", ctypes.c_void_p), ("leak_base", ctypes.c_void_p), ("leak", ctypes.c_void_p),
        ("n_gates", ctypes.c_int64), ("n_nets", ctypes.c_int64),
        ("gate_cell", ctypes.c_void_p), ("gate_out_net", ctypes.c_void_p), ("gate_init", ctypes.c_void_p),
        ("net_load", ctypes.c_void_p), ("leak_scale", ctypes.c_void_p),
        ("n_events", ctypes.c_int64), ("gate_off", ctypes.c_void_p), ("t", ctypes.c_void_p),
        ("pin_bit", ctypes.c_void_p), ("slew", ctypes.c_void_p),
        ("t_end", ctypes.c_int64), ("bin_ps", ctypes.c_int64), ("vdd", ctypes.c_double),
        ("sw_mode", ctypes.c_int32), ("state_all_pins", ctypes.c_int32), ("glitch_clk", ctypes.c_int64),
        ("n_tpat", ctypes.c_void_p), ("tpat_base", ctypes.c_void_p), ("tpat_care", ctypes.c_void_p),
        ("tpat_value", ctypes.c_void_p), ("tpat_table", ctypes.c_void_p), ("n_lpat", ctypes.c_void_p),
        ("lpat_base", ctypes.c_void_p), ("lpat_care", ctypes.c_void_p), ("lpat_value", ctypes.c_void_p),
        ("lpat_leak", ctypes.c_void_p),
    ]

_PATTERNS = (("n_tpat", np.int32), ("tpat_base", np.int64), ("tpat_care", np.uint32), ("tpat_value", np.uint32),
             ("tpat_table", np.int16), ("n_lpat", np.int32), ("lpat_base", np.int64), ("lpat_care", np.uint32),
             ("lpat_value", np.uint32), ("lpat_leak", np.float32))


def build(force: bool = True, plant: int = 0, out: Optional[str] = None) -> str:
    """Compile the oracle (gcc, OpenMP). plant>0 builds a deliberately wrong
    variant (for the tests that check the pins catch mistakes)."""
    out = out or _SO
    if force or not os.path.exists(out):
        tmp = out + ".tmp"
        cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, os.path.join(_HERE, "oracle.c"), "-lm"]
        if plant:
            cmd.insert(1, f"-DORC_PLANT={plant}")
        subprocess.check_call(cmd)
        os.replace(tmp, out)
    return out


class Oracle:
    def __init__(self, so_path: Optional[str] = None):
        path = so_path or _SO
        if so_path is None and not os.path.exists(path):
            build()
        self.lib = ctypes.CDLL(path)
        L = self.lib
        L.orc_forward.restype = ctypes.c_int
        L.orc_forward.argtypes = [ctypes.POINTER(_Problem), ctypes.c_int64, ctypes.c_int64, ctypes.c_int,
                                  ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                  ctypes.POINTER(ctypes.c_int64)]
        L.orc_event_trace.argtypes = [ctypes.POINTER(_Problem), ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.POINTER(ctypes.c_int64)]
        L.orc_adjoint.argtypes = [ctypes.POINTER(_Problem), ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                  ctypes.c_void_p, ctypes.c_int]
        L.orc_validate.argtypes = [ctypes.POINTER(_Problem), ctypes.POINTER(ctypes.c_int64)]
        L.orc_gate_report.argtypes = [ctypes.POINTER(_Problem), ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64),
                                      ctypes.c_int]
        L.orc_bilerp.restype = ctypes.c_double
        L.orc_bilerp.argtypes = [ctypes.POINTER(_Problem), ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                 ctypes.c_double]
        L.orc_num_bins.restype = ctypes.c_int64
        L.orc_num_bins.argtypes = [ctypes.POINTER(_Problem)]
        L.orc_max_threads.restype = ctypes.c_int
        L.orc_pattern_scan.restype = ctypes.c_int64
        L.orc_pattern_scan.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32]

    # -- marshalling -------------------------------------------------------
    @staticmethod
    def _arrays(prob, net_load=None, leak_scale=None):
        lib, net, ev = prob.lib, prob.net, prob.ev
        keep = dict(
            n_inputs=np.ascontiguousarray(lib.n_inputs, np.int32),
            slew_axis=np.ascontiguousarray(lib.slew_axis, np.float32),
            load_axis=np.ascontiguousarray(lib.load_axis, np.float32),
            map_base=np.ascontiguousarray(lib.map_base, np.int64),
            state_to_table=np.ascontiguousarray(lib.state_to_table, np.int16),
            table_base=np.ascontiguousarray(lib.table_base, np.int64),
            tables=np.ascontiguousarray(lib.tables, np.float32),
            leak_base=np.ascontiguousarray(lib.leak_base, np.int64),
            leak=np.ascontiguousarray(lib.leak, np.float32),
            gate_cell=np.ascontiguousarray(net.gate_cell, np.int32),
            gate_out_net=np.ascontiguousarray(net.gate_out_net, np.int32),
            gate_init=np.ascontiguousarray(net.gate_init, np.uint32),
            net_load=np.ascontiguousarray(net.net_load if net_load is None else net_load, np.float32),
            leak_scale=np.ascontiguousarray(net.leak_scale if leak_scale is None else leak_scale, np.float32),
            gate_off=np.ascontiguousarray(ev.gate_off, np.int64),
            t=np.ascontiguousarray(ev.t, np.int64),
            pin_bit=np.ascontiguousarray(ev.pin_bit, np.uint8),
            slew=np.ascontiguousarray(ev.slew, np.float32),
        )
        if getattr(lib, "n_tpat", None) is not None:
            for name, dt in _PATTERNS:
                keep[name] = np.ascontiguousarray(getattr(lib, name), dt)
        P = _Problem()
        P.n_cells, P.n_slew, P.n_load = lib.n_cells, lib.n_slew, lib.n_load
        for k, a in keep.items():
            setattr(P, k, a.ctypes.data)
        P.n_gates, P.n_nets = net.n_gates, net.n_nets
        P.n_events = ev.n_events
        P.t_end, P.bin_ps, P.vdd, P.sw_mode = ev.t_end, prob.bin_ps, prob.vdd, prob.sw_mode
        P.state_all_pins = int(getattr(prob, "state_all_pins", 0))
        P.glitch_clk = int(getattr(prob, "glitch_clk", 0))
        return P, keep

    # -- API ---------------------------------------------------------------
    def num_bins(self, prob) -> int:
        return -(-prob.ev.t_end // prob.bin_ps)

    def forward(self, prob, b0: int = 0, b1: Optional[int] = None, leak_mode: int = 1,
                gates: Optional[Sequence[int]] = None, net_load=None, leak_scale=None, nthreads: int = 0,
                return_totals: bool = False):
        """Binned energy E[b0:b1] (fJ) in FP64; power is E / bin_ps (mW)."""
        P, keep = self._arrays(prob, net_load, leak_scale)
        nb = self.num_bins(prob)
        b1 = nb if b1 is None else b1
        E = np.zeros(max(0, b1 - b0), np.float64)
        tot = np.zeros(4, np.float64)
        gl = None if gates is None else np.ascontiguousarray(gates, np.int64)
        bad = ctypes.c_int64(-1)
        rc = self.lib.orc_forward(ctypes.byref(P), b0, b1, leak_mode, None if gl is None else gl.ctypes.data,
                                  0 if gl is None else len(gl), E.ctypes.data, tot.ctypes.data, nthreads,
                                  ctypes.byref(bad))
        if rc != OK:
            raise OracleError(rc, bad.value)
        return (E, tot) if return_totals else E

    def power(self, prob, **kw):
        """P_b in mW (FP64)."""
        return self.forward(prob, **kw) / float(prob.bin_ps)

    def event_trace(self, prob):
        P, keep = self._arrays(prob)
        st = np.zeros(prob.ev.n_events, np.int32)
        b = np.zeros(prob.ev.n_events, np.int64)
        bad = ctypes.c_int64(-1)
        rc = self.lib.orc_event_trace(ctypes.byref(P), st.ctypes.data, b.ctypes.data, ctypes.byref(bad))
        if rc != OK:
            raise OracleError(rc, bad.value)
        return st, b

    def gate_report(self, prob, net_load=None, leak_scale=None, nthreads: int = 0):
        """(per-gate energies [n_gates, 4] in fJ: leakage, internal, switching,
        glitch; t_max = latest event time, -1 without events)."""
        P, keep = self._arrays(prob, net_load, leak_scale)
        ge = np.zeros((prob.net.n_gates, 4), np.float64)
        tm = ctypes.c_int64(-1)
        rc = self.lib.orc_gate_report(ctypes.byref(P), ge.ctypes.data, ctypes.byref(tm), nthreads)
        if rc != OK:
            raise OracleError(rc)
        return ge, tm.value

    def validate(self, prob):
        P, keep = self._arrays(prob)
        bad = ctypes.c_int64(-1)
        rc = self.lib.orc_validate(ctypes.byref(P), ctypes.byref(bad))
        return rc, bad.value

    def adjoint(self, prob, gP: np.ndarray, leak_mode: int = 1, net_load=None, leak_scale=None, nthreads: int = 0):
        P, keep = self._arrays(prob, net_load, leak_scale)
        gP = np.ascontiguousarray(gP, np.float64)
        assert gP.shape[0] == self.num_bins(prob)
        gl = np.zeros(prob.net.n_nets, np.float64)
        gs = np.zeros(prob.net.n_gates, np.float64)
        rc = self.lib.orc_adjoint(ctypes.byref(P), gP.ctypes.data, leak_mode, gl.ctypes.data, gs.ctypes.data,
                                  nthreads)
        if rc != OK:
            raise OracleError(rc)
        return gl, gs

    def bilerp(self, prob, cell: int, table: int, slew: float, load: float) -> float:
        P, keep = self._arrays(prob)
        return self.lib.orc_bilerp(ctypes.byref(P), cell, table, slew, load)

    def pattern_scan(self, care, value, s: int) -> int:
        """First pattern whose care pins agree with state s, -1 if none."""
        care = np.ascontiguousarray(care, np.uint32)
        value = np.ascontiguousarray(value, np.uint32)
        return int(self.lib.orc_pattern_scan(len(care), care.ctypes.data, value.ctypes.data, int(s)))

    def max_threads(self) -> int:
        return self.lib.orc_max_threads()


_default: Optional[Oracle] = None


def get() -> Oracle:
    global _default
    if _default is None:
        _default = Oracle()
    return _default


def lse_loss_grad(P: np.ndarray, beta: float):
    """Smooth peak-power loss L = (1/beta) log sum_b exp(beta P_b) in FP64
    with the max shift, and dL/dP_b = softmax(beta P)_b."""
    P = np.asarray(P, np.float64)
    m = P.max()
    w = np.exp(beta * (P - m))
    s = w.sum()
    return m + np.log(s) / beta, w / s
