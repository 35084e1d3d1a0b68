"""gtpower: binned gate-level power waveforms on MI355X (gfx950).

A thin ctypes binding over the C ABI in ``include/gtpower.h`` (argument
marshalling only; every step runs in the library's HIP kernels). PyTorch
provides device memory and the stream. The library must be built first
(``build()`` or ``__graft_entry__.build()``); importing never falls back to
any other implementation.

    ctx = Context(device=0)
    ctx.load_library(lib)                     # host arrays (see Context.load_library)
    ctx.load_netlist(gate_cell, gate_out, gate_init, n_nets)   # device int32/uint32 tensors
    ctx.load_events(gate_off, t, pin_bit, slew, t_end)         # device tensors (borrowed)
    ctx.set_params(vdd=0.8, bin_ps=50)
    P = ctx.forward(net_load, leak_scale)     # FP32 mW per bin
    P = binned_power(ctx, net_load, leak_scale)   # differentiable (BinnedPower)
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_ROOT = os.path.dirname(_HERE)
SO_PATH = os.path.join(_HERE, "libgtpower.so")
_SRCS = [os.path.join(_HERE, "csrc", "gtpower.hip"), os.path.join(_HERE, "csrc", "gtp_pack.hip")]

HIPCC_FLAGS = ["-O3", "--offload-arch=gfx950", "-std=c++17", "-shared", "-fPIC",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]

STATUS = {0: "OK", 1: "INVALID_ARG", 2: "OUT_OF_MEMORY", 3: "HIP", 4: "NOT_LOADED", 5: "EVENT_ORDER",
          6: "EVENT_RANGE", 7: "NOT_TOGGLE", 8: "UNSUPPORTED", 9: "SCALE_RANGE", 10: "LOAD_RANGE"}

ABI_SYMBOLS = ["gtp_create", "gtp_destroy", "gtp_set_stream", "gtp_last_error", "gtp_sync", "gtp_load_library",
               "gtp_load_netlist", "gtp_load_events", "gtp_bad_event", "gtp_set_params", "gtp_num_bins",
               "gtp_set_tuning", "gtp_get_tuning", "gtp_plan_info", "gtp_autotune", "gtp_load_traces",
               "gtp_batch_bins", "gtp_forward_batched", "gtp_forward_trace", "gtp_forward", "gtp_adjoint", "gtp_debug_event_trace",
               "gtp_device_bytes", "gtp_profile_enable", "gtp_profile_read", "gtp_fixed_point_bits",
               "gtp_forward_noalloc", "gtp_gate_report", "gtp_expand_when", "gtp_stream_begin", "gtp_stream_push",
               "gtp_stream_step", "gtp_stream_end"]


def build(out: Optional[str] = None) -> str:
    """Compile libgtpower.so for gfx950 in-tree with hipcc (always recompiles)."""
    out = out or SO_PATH
    tmp = out + ".tmp"
    cmd = ["hipcc", *HIPCC_FLAGS, "-o", tmp, *_SRCS]
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


class GtpError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"gtpower {STATUS.get(code, code)}: {msg}")
        self.code = code
        self.status = STATUS.get(code, str(code))


class _Library(ctypes.Structure):
    _fields_ = [("n_cells", ctypes.c_int32), ("n_slew", ctypes.c_int32), ("n_load", ctypes.c_int32),
                ("n_inputs", ctypes.c_void_p), ("slew_axis_ps", ctypes.c_void_p), ("load_axis_ff", ctypes.c_void_p),
                ("map_base", ctypes.c_void_p), ("state_to_table", ctypes.c_void_p), ("table_base", ctypes.c_void_p),
                ("tables_fj", ctypes.c_void_p), ("leak_base", ctypes.c_void_p), ("leak_nw", ctypes.c_void_p),
                ("n_map", ctypes.c_int64), ("n_tables", ctypes.c_int64), ("n_leak", ctypes.c_int64),
                ("all_pin_state", ctypes.c_int32),
                ("n_tpat", ctypes.c_void_p), ("tpat_base", ctypes.c_void_p), ("tpat_care", ctypes.c_void_p),
                ("tpat_value", ctypes.c_void_p), ("tpat_table", ctypes.c_void_p), ("n_lpat", ctypes.c_void_p),
                ("lpat_base", ctypes.c_void_p), ("lpat_care", ctypes.c_void_p), ("lpat_value", ctypes.c_void_p),
                ("lpat_leak_nw", ctypes.c_void_p), ("n_tpat_total", ctypes.c_int64), ("n_lpat_total", ctypes.c_int64)]

# state-pattern fields of a library object (all optional; n_tpat None: none)
_PATTERN_FIELDS = (("n_tpat", np.int32), ("tpat_base", np.int64), ("tpat_care", np.uint32),
                   ("tpat_value", np.uint32), ("tpat_table", np.int16), ("n_lpat", np.int32),
                   ("lpat_base", np.int64), ("lpat_care", np.uint32), ("lpat_value", np.uint32),
                   ("lpat_leak", np.float32))


class _Events(ctypes.Structure):
    _fields_ = [("n_events", ctypes.c_int64), ("t_end_ps", ctypes.c_int64), ("gate_off", ctypes.c_void_p),
                ("t_ps", ctypes.c_void_p), ("pin_bit", ctypes.c_void_p), ("slew_ps", ctypes.c_void_p)]


class _Params(ctypes.Structure):
    _fields_ = [("vdd", ctypes.c_double), ("bin_ps", ctypes.c_int64), ("glitch_clk_ps", ctypes.c_int64),
                ("sw_mode", ctypes.c_int32)]


class _Tuning(ctypes.Structure):
    _fields_ = [("algo", ctypes.c_int32), ("bins_per_tile_log2", ctypes.c_int32), ("tile_threads", ctypes.c_int32),
                ("unit_events", ctypes.c_int32), ("gate_block_log2", ctypes.c_int32)]


class _PlanStats(ctypes.Structure):
    _fields_ = [("n_events_packed", ctypes.c_int64), ("n_units", ctypes.c_int64), ("n_groups", ctypes.c_int64),
                ("n_tiles", ctypes.c_int32), ("tile_log2", ctypes.c_int32), ("max_tile_groups", ctypes.c_int32),
                ("packed_bytes", ctypes.c_int64), ("pack_ms", ctypes.c_double), ("lane_steps", ctypes.c_int64)]


class _Range(ctypes.Structure):
    _fields_ = [("max_bin_events", ctypes.c_int64), ("bin_ps", ctypes.c_int64), ("event_energy_fj", ctypes.c_double),
                ("leak_rate_fj_per_ps", ctypes.c_double), ("leak_value_nw", ctypes.c_double)]


def fixed_point_bits(max_bin_events: int, bin_ps: int, event_energy_fj: float, leak_rate_fj_per_ps: float,
                     leak_value_nw: float) -> int:
    """Fixed-point exponent m the library uses for these bounds (gtp_fixed_point_bits)."""
    L = load_library()
    r = _Range(int(max_bin_events), int(bin_ps), float(event_energy_fj), float(leak_rate_fj_per_ps),
               float(leak_value_nw))
    m = ctypes.c_int32()
    rc = L.gtp_fixed_point_bits(ctypes.byref(r), ctypes.byref(m))
    if rc != 0:
        raise GtpError(rc, "fixed-point range")
    return m.value


def _host(a, dtype):
    """(address, length, keep-alive) of a host array: a numpy array or a CPU
    tensor (pinned or not) of the given dtype, contiguous."""
    if hasattr(a, "data_ptr"):
        if a.device.type != "cpu" or not a.is_contiguous():
            raise ValueError("stream windows are contiguous host arrays")
        if a.element_size() != np.dtype(dtype).itemsize:
            raise ValueError(f"window array of element size {a.element_size()}, want {np.dtype(dtype).itemsize}")
        return a.data_ptr(), a.numel(), a
    a = np.ascontiguousarray(a, dtype)
    return a.ctypes.data, a.size, a


def expand_when(n_pins: int, care, value, item, default_item: int) -> np.ndarray:
    """Per-state item array of state patterns with don't-care pins
    (gtp_expand_when): entry s holds the item of the first pattern whose
    care bits agree with s, default_item where none does."""
    L = load_library()
    care = np.ascontiguousarray(care, np.uint32)
    value = np.ascontiguousarray(value, np.uint32)
    item = np.ascontiguousarray(item, np.int32)
    if not (care.shape == value.shape == item.shape) or care.ndim != 1:
        raise ValueError("care, value and item must be 1-D arrays of one length")
    if not 0 <= int(n_pins) <= 16:
        raise ValueError("n_pins must lie in 0..16")
    out = np.empty(1 << int(n_pins), np.int32)
    rc = L.gtp_expand_when(int(n_pins), len(care), care.ctypes.data, value.ctypes.data, item.ctypes.data,
                           int(default_item), out.ctypes.data)
    if rc != 0:
        raise GtpError(rc, "state-pattern expansion")
    return out


_lib = None


def load_library(path: Optional[str] = None):
    """Load libgtpower.so (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or SO_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"{p} is not built: run paper_2609_05960_amd.build() (no CPU fallback exists)")
    # torch's HIP runtime first: the library then binds to that same runtime
    # (its stream handles are torch's). Loaded the other way round, the
    # process would hold two HIP runtimes and the library would see no device.
    import torch  # noqa: F401
    L = ctypes.CDLL(p)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
    sig = {
        "gtp_create": [ctypes.POINTER(vp), i32, vp], "gtp_destroy": [vp], "gtp_set_stream": [vp, vp],
        "gtp_sync": [vp], "gtp_load_library": [vp, ctypes.POINTER(_Library)],
        "gtp_load_netlist": [vp, i64, i64, vp, vp, vp], "gtp_load_events": [vp, ctypes.POINTER(_Events), i32],
        "gtp_set_params": [vp, ctypes.POINTER(_Params)], "gtp_num_bins": [vp, ctypes.POINTER(i64)],
        "gtp_set_tuning": [vp, ctypes.POINTER(_Tuning)], "gtp_get_tuning": [vp, ctypes.POINTER(_Tuning)],
        "gtp_plan_info": [vp, ctypes.POINTER(_PlanStats)],
        "gtp_autotune": [vp, ctypes.c_char_p],
        "gtp_load_traces": [vp, i32, ctypes.POINTER(_Events), i32],
        "gtp_batch_bins": [vp, ctypes.POINTER(i64), ctypes.POINTER(i64)],
        "gtp_forward_batched": [vp, vp, vp, vp, i32],
        "gtp_forward_trace": [vp, i32, vp, vp, vp],
        "gtp_forward": [vp, vp, vp, vp], "gtp_adjoint": [vp, vp, vp, vp, vp, vp],
        "gtp_forward_noalloc": [vp, vp, vp, vp],
        "gtp_gate_report": [vp, vp, vp, vp, vp, vp],
        "gtp_debug_event_trace": [vp, vp, vp],
        "gtp_fixed_point_bits": [ctypes.POINTER(_Range), ctypes.POINTER(ctypes.c_int32)],
        "gtp_expand_when": [i32, i32, vp, vp, vp, i32, vp],
        "gtp_stream_begin": [vp, i64, i32], "gtp_stream_push": [vp, ctypes.POINTER(_Events), i64, i64],
        "gtp_stream_step": [vp, vp, vp, vp], "gtp_stream_end": [vp],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    L.gtp_last_error.argtypes = [vp]
    L.gtp_last_error.restype = ctypes.c_char_p
    L.gtp_bad_event.argtypes = [vp]
    L.gtp_bad_event.restype = i64
    L.gtp_device_bytes.argtypes = [vp]
    L.gtp_device_bytes.restype = i64
    L.gtp_profile_enable.argtypes = [vp, i32]
    L.gtp_profile_enable.restype = ctypes.c_int
    L.gtp_profile_read.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(i64),
                                   ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32)]
    L.gtp_profile_read.restype = ctypes.c_int
    if path is None:
        _lib = L
    return L


def _dptr(x) -> Optional[int]:
    if x is None:
        return None
    return x.data_ptr()


def _np(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


class Context:
    """One library context on a HIP device (not thread-safe)."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self.torch = torch
        self.L = load_library()
        self.device = torch.device("cuda", device)
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        self._chk(self.L.gtp_create(ctypes.byref(h), device, ctypes.c_void_p(s.cuda_stream)), None)
        self.h = h
        self._keep = {}
        self.n_gates = self.n_nets = self.n_events = 0
        self.n_bins = 0

    def _chk(self, rc, h="self"):
        if rc != 0:
            handle = self.h if h == "self" else None
            msg = self.L.gtp_last_error(handle).decode() if handle else ""
            raise GtpError(rc, msg)

    def close(self):
        if getattr(self, "h", None):
            self.L.gtp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream):
        self._chk(self.L.gtp_set_stream(self.h, ctypes.c_void_p(stream.cuda_stream)))

    def sync(self):
        self._chk(self.L.gtp_sync(self.h))

    # -- loading ------------------------------------------------------------
    def load_library(self, lib, all_pin_state: int = 0):
        """lib: object with n_cells, n_slew, n_load and host arrays n_inputs,
        slew_axis, load_axis, map_base, state_to_table, table_base, tables,
        leak_base, leak (the layout of include/gtpower.h gtp_library), and
        optionally the state patterns n_tpat, tpat_base, tpat_care,
        tpat_value, tpat_table, n_lpat, lpat_base, lpat_care, lpat_value,
        lpat_leak (n_tpat None or absent: none); all_pin_state = 1: its
        states cover every pin (bit I = the output)."""
        arrs = dict(n_inputs=_np(lib.n_inputs, np.int32), slew=_np(lib.slew_axis, np.float32),
                    load=_np(lib.load_axis, np.float32), map_base=_np(lib.map_base, np.int64),
                    s2t=_np(lib.state_to_table, np.int16), table_base=_np(lib.table_base, np.int64),
                    tables=_np(lib.tables, np.float32), leak_base=_np(lib.leak_base, np.int64),
                    leak=_np(lib.leak, np.float32))
        S = _Library()
        S.n_cells, S.n_slew, S.n_load = int(lib.n_cells), int(lib.n_slew), int(lib.n_load)
        S.n_inputs, S.slew_axis_ps, S.load_axis_ff = (arrs[k].ctypes.data for k in ("n_inputs", "slew", "load"))
        S.map_base, S.state_to_table, S.table_base = (arrs[k].ctypes.data for k in ("map_base", "s2t", "table_base"))
        S.tables_fj, S.leak_base, S.leak_nw = (arrs[k].ctypes.data for k in ("tables", "leak_base", "leak"))
        S.n_map = arrs["s2t"].size
        S.n_tables = arrs["tables"].size // (S.n_slew * S.n_load)
        S.n_leak = arrs["leak"].size
        S.all_pin_state = int(all_pin_state)
        if getattr(lib, "n_tpat", None) is not None:
            for name, dt in _PATTERN_FIELDS:
                arrs[name] = _np(getattr(lib, name), dt)
            for name in ("n_tpat", "tpat_base", "tpat_care", "tpat_value", "tpat_table", "n_lpat", "lpat_base",
                         "lpat_care", "lpat_value"):
                setattr(S, name, arrs[name].ctypes.data)
            S.lpat_leak_nw = arrs["lpat_leak"].ctypes.data
            S.n_tpat_total = arrs["tpat_care"].size
            S.n_lpat_total = arrs["lpat_care"].size
        self._chk(self.L.gtp_load_library(self.h, ctypes.byref(S)))

    def load_netlist(self, gate_cell, gate_out_net, gate_init, n_nets: int):
        t = self.torch
        gc = gate_cell.to(self.device, t.int32).contiguous()
        go = gate_out_net.to(self.device, t.int32).contiguous()
        gi = gate_init.to(self.device, t.int32).contiguous()
        self._chk(self.L.gtp_load_netlist(self.h, gc.numel(), int(n_nets), _dptr(gc), _dptr(go), _dptr(gi)))
        self.n_gates, self.n_nets = gc.numel(), int(n_nets)

    def load_events(self, gate_off, t_ps, pin_bit, slew_ps, t_end: int, validate: bool = False):
        """Device tensors: gate_off int64 [G+1], t int64, pin_bit uint8, slew
        float32. They are borrowed: this object keeps references to them."""
        t = self.torch
        for x, dt in ((gate_off, t.int64), (t_ps, t.int64), (pin_bit, t.uint8), (slew_ps, t.float32)):
            if x.dtype != dt or not x.is_contiguous() or x.device != self.device:
                raise ValueError(f"event tensors must be contiguous {dt} on {self.device}")
        E = _Events()
        E.n_events, E.t_end_ps = t_ps.numel(), int(t_end)
        E.gate_off, E.t_ps, E.pin_bit, E.slew_ps = _dptr(gate_off), _dptr(t_ps), _dptr(pin_bit), _dptr(slew_ps)
        self._keep["events"] = (gate_off, t_ps, pin_bit, slew_ps)
        rc = self.L.gtp_load_events(self.h, ctypes.byref(E), 1 if validate else 0)
        if rc != 0:
            err = GtpError(rc, self.L.gtp_last_error(self.h).decode())
            err.bad_event = self.L.gtp_bad_event(self.h)
            raise err
        self.n_events = t_ps.numel()
        self.t_end = int(t_end)
        n = ctypes.c_int64()
        if self.L.gtp_num_bins(self.h, ctypes.byref(n)) == 0:
            self.n_bins = n.value

    def set_params(self, vdd: float = 0.8, bin_ps: int = 50, sw_mode: int = 0, glitch_clk_ps: int = 0):
        p = _Params(float(vdd), int(bin_ps), int(glitch_clk_ps), int(sw_mode))
        self._chk(self.L.gtp_set_params(self.h, ctypes.byref(p)))
        self.n_bins = 0
        if "events" in self._keep:
            n = ctypes.c_int64()
            self._chk(self.L.gtp_num_bins(self.h, ctypes.byref(n)))
            self.n_bins = n.value
        self.vdd, self.bin_ps, self.sw_mode, self.glitch_clk_ps = float(vdd), int(bin_ps), int(sw_mode), int(glitch_clk_ps)

    def set_tuning(self, algo: int = 0, bins_per_tile_log2: int = 0, tile_threads: int = 0, unit_events: int = 0,
                   gate_block_log2: int = 0):
        tu = _Tuning(int(algo), int(bins_per_tile_log2), int(tile_threads), int(unit_events), int(gate_block_log2))
        self._chk(self.L.gtp_set_tuning(self.h, ctypes.byref(tu)))

    def get_tuning(self):
        tu = _Tuning()
        self._chk(self.L.gtp_get_tuning(self.h, ctypes.byref(tu)))
        return {k: getattr(tu, k) for k, _ in _Tuning._fields_}

    def autotune(self, cache_path: Optional[str] = None):
        """Pick the fastest tuning for the loaded events (or batch); see gtp_autotune."""
        self._chk(self.L.gtp_autotune(self.h, cache_path.encode() if cache_path else None))
        return self.get_tuning()

    # -- batched traces -------------------------------------------------------
    def load_traces(self, traces, validate: bool = False):
        """traces: list of (gate_off, t_ps, pin_bit, slew_ps, t_end) device tensors
        (borrowed; this object keeps references)."""
        t = self.torch
        arr = (_Events * len(traces))()
        keep = []
        for i, (go, tp, pb, sl, t_end) in enumerate(traces):
            for x, dt in ((go, t.int64), (tp, t.int64), (pb, t.uint8), (sl, t.float32)):
                if x.dtype != dt or not x.is_contiguous() or x.device != self.device:
                    raise ValueError(f"event tensors must be contiguous {dt} on {self.device}")
            arr[i].n_events, arr[i].t_end_ps = tp.numel(), int(t_end)
            arr[i].gate_off, arr[i].t_ps, arr[i].pin_bit, arr[i].slew_ps = (_dptr(go), _dptr(tp), _dptr(pb),
                                                                            _dptr(sl))
            keep.append((go, tp, pb, sl))
        self._keep["traces"] = keep
        rc = self.L.gtp_load_traces(self.h, len(traces), arr, 1 if validate else 0)
        if rc != 0:
            err = GtpError(rc, self.L.gtp_last_error(self.h).decode())
            err.bad_event = self.L.gtp_bad_event(self.h)
            raise err
        self.n_traces = len(traces)

    def batch_bins(self):
        """(total bins, offsets[n_traces + 1]) of the concatenated batched output."""
        tot = ctypes.c_int64()
        offs = (ctypes.c_int64 * (self.n_traces + 1))()
        self._chk(self.L.gtp_batch_bins(self.h, ctypes.byref(tot), offs))
        return tot.value, np.array(offs[:], dtype=np.int64)

    def forward_batched(self, net_load, leak_scale=None, out=None, use_graph: bool = False):
        net_load = self._vec(net_load, self.n_nets, "net_load")
        leak_scale = self._vec(leak_scale, self.n_gates, "leak_scale")
        tot, _ = self.batch_bins()
        out = self._out(out, tot)
        self._chk(self.L.gtp_forward_batched(self.h, _dptr(net_load), _dptr(leak_scale), _dptr(out),
                                             1 if use_graph else 0))
        return out

    def forward_trace(self, i: int, net_load, leak_scale=None, out=None):
        net_load = self._vec(net_load, self.n_nets, "net_load")
        leak_scale = self._vec(leak_scale, self.n_gates, "leak_scale")
        _, offs = self.batch_bins()
        out = self._out(out, int(offs[i + 1] - offs[i]))
        self._chk(self.L.gtp_forward_trace(self.h, int(i), _dptr(net_load), _dptr(leak_scale), _dptr(out)))
        return out

    def plan_info(self) -> dict:
        """Statistics of the packed layout (built on demand; synchronises)."""
        ps = _PlanStats()
        self._chk(self.L.gtp_plan_info(self.h, ctypes.byref(ps)))
        return {k: getattr(ps, k) for k, _ in _PlanStats._fields_}

    def device_bytes(self) -> int:
        return self.L.gtp_device_bytes(self.h)

    def profile(self, enable: bool = True):
        """Start (clearing earlier records) or stop per-kernel HIP-event timing."""
        self._chk(self.L.gtp_profile_enable(self.h, 1 if enable else 0))

    def profile_read(self):
        """{kernel name: (launches, total ms)} since profile(True)."""
        cap = 64
        names = (ctypes.c_char_p * cap)()
        cnt = (ctypes.c_int64 * cap)()
        ms = (ctypes.c_double * cap)()
        n = ctypes.c_int32()
        self._chk(self.L.gtp_profile_read(self.h, cap, names, cnt, ms, ctypes.byref(n)))
        return {names[i].decode(): (cnt[i], ms[i]) for i in range(min(n.value, cap))}

    # -- compute ------------------------------------------------------------
    def _vec(self, x, n, name):
        t = self.torch
        if x is None:
            return None
        if x.dtype != t.float32 or x.device != self.device or not x.is_contiguous() or x.numel() != n:
            raise ValueError(f"{name} must be a contiguous float32 tensor of {n} elements on {self.device}")
        return x

    def _out(self, out, n):
        t = self.torch
        if out is None:
            return t.empty(n, dtype=t.float32, device=self.device)
        if out.dtype != t.float32 or out.device != self.device or not out.is_contiguous() or out.numel() < n:
            raise ValueError(f"out must be a contiguous float32 tensor of at least {n} elements on {self.device}")
        return out

    def forward(self, net_load, leak_scale=None, out=None):
        net_load = self._vec(net_load, self.n_nets, "net_load")
        leak_scale = self._vec(leak_scale, self.n_gates, "leak_scale")
        out = self._out(out, self.n_bins)
        self._chk(self.L.gtp_forward(self.h, _dptr(net_load), _dptr(leak_scale), _dptr(out)))
        return out

    # -- streamed windows ----------------------------------------------------
    def stream_begin(self, t_end: int, validate: bool = False):
        """gtp_stream_begin: evaluate one trace of t_end ps window by window;
        returns the FP32 power tensor of the whole trace the steps fill."""
        self._chk(self.L.gtp_stream_begin(self.h, int(t_end), 1 if validate else 0))
        self._stream = {"n_bins": -(-int(t_end) // self.bin_ps), "pending": []}
        t = self.torch
        return t.empty(self._stream["n_bins"], dtype=t.float32, device=self.device)

    def stream_push(self, gate_off, t_ps, pin_bit, slew_ps, t0: int, t1: int):
        """gtp_stream_push: host arrays of the window [t0, t1) (numpy, or
        pinned CPU tensors); kept alive here until their window is stepped."""
        arrs = [_host(a, dt) for a, dt in ((gate_off, np.int64), (t_ps, np.int64), (pin_bit, np.uint8),
                                           (slew_ps, np.float32))]
        E = _Events()
        E.n_events, E.t_end_ps = int(arrs[1][1]), int(t1)
        E.gate_off, E.t_ps, E.pin_bit, E.slew_ps = (a[0] for a in arrs)
        self._chk(self.L.gtp_stream_push(self.h, ctypes.byref(E), int(t0), int(t1)))
        self._stream["pending"].append(arrs)

    def stream_step(self, net_load, leak_scale, out):
        """gtp_stream_step: evaluate the oldest pushed window into out."""
        net_load = self._vec(net_load, self.n_nets, "net_load")
        leak_scale = self._vec(leak_scale, self.n_gates, "leak_scale")
        out = self._out(out, self._stream["n_bins"])
        try:
            self._chk(self.L.gtp_stream_step(self.h, _dptr(net_load), _dptr(leak_scale), _dptr(out)))
        finally:
            if self._stream["pending"]:
                self._stream["pending"].pop(0)
        return out

    def stream_end(self):
        self._chk(self.L.gtp_stream_end(self.h))
        self._stream = None

    def forward_noalloc(self, net_load, leak_scale=None, out=None):
        """gtp_forward_noalloc: the forward without device allocation (the packed
        layout must be built first, e.g. by plan_info(); out must be given by
        callers that cannot allocate)."""
        net_load = self._vec(net_load, self.n_nets, "net_load")
        leak_scale = self._vec(leak_scale, self.n_gates, "leak_scale")
        out = self._out(out, self.n_bins)
        self._chk(self.L.gtp_forward_noalloc(self.h, _dptr(net_load), _dptr(leak_scale), _dptr(out)))
        return out

    def adjoint(self, net_load, leak_scale, grad_power):
        net_load = self._vec(net_load, self.n_nets, "net_load")
        leak_scale = self._vec(leak_scale, self.n_gates, "leak_scale")
        grad_power = self._vec(grad_power, self.n_bins, "grad_power")
        t = self.torch
        gl = t.empty(self.n_nets, dtype=t.float32, device=self.device)
        gs = t.empty(self.n_gates, dtype=t.float32, device=self.device)
        self._chk(self.L.gtp_adjoint(self.h, _dptr(net_load), _dptr(leak_scale), _dptr(grad_power), _dptr(gl),
                                     _dptr(gs)))
        return gl, gs

    def report(self, net_load, leak_scale=None, power=None):
        """gtp_gate_report: per-gate energies [n_gates, 4] (FP64 fJ: leakage,
        internal, switching, glitch) and the design summary (totals, latest
        event time, peak of `power`, the paper's averages E / t_max and the
        window average)."""
        net_load = self._vec(net_load, self.n_nets, "net_load")
        leak_scale = self._vec(leak_scale, self.n_gates, "leak_scale")
        if power is not None:
            power = self._vec(power, self.n_bins, "power")
        t = self.torch
        ge = t.empty((self.n_gates, 4), dtype=t.float64, device=self.device)
        tot = (ctypes.c_double * 12)()
        self._chk(self.L.gtp_gate_report(self.h, _dptr(net_load), _dptr(leak_scale), _dptr(power), _dptr(ge),
                                         ctypes.cast(tot, ctypes.c_void_p)))
        v = list(tot)
        keys = ("leak", "int", "sw", "gl")
        return ge, {"energy_fj": dict(zip(keys, v[0:4])), "t_max_ps": v[4], "peak_mw": v[5],
                    "avg_mw_tmax": dict(zip(keys, v[6:10])), "avg_mw_window": v[10], "t_end_ps": v[11]}

    def event_trace(self):
        t = self.torch
        st = t.empty(self.n_events, dtype=t.int32, device=self.device)
        b = t.empty(self.n_events, dtype=t.int64, device=self.device)
        self._chk(self.L.gtp_debug_event_trace(self.h, _dptr(st), _dptr(b)))
        return st, b


def _binned_power_fn():
    import torch

    class BinnedPower(torch.autograd.Function):
        """P = forward(net_load, leak_scale); backward through the library's
        adjoint kernel. Event times and states are context, not inputs."""

        @staticmethod
        def forward(actx, ctx: Context, net_load, leak_scale):
            P = ctx.forward(net_load.detach().contiguous(), leak_scale.detach().contiguous())
            actx.gtp = ctx
            actx.save_for_backward(net_load, leak_scale)
            return P

        @staticmethod
        def backward(actx, grad_P):
            net_load, leak_scale = actx.saved_tensors
            gl, gs = actx.gtp.adjoint(net_load.detach().contiguous(), leak_scale.detach().contiguous(),
                                      grad_P.detach().to(torch.float32).contiguous())
            return None, gl, gs

    return BinnedPower


_BP = None


def binned_power(ctx: Context, net_load, leak_scale):
    """Differentiable binned power (FP32 mW per bin)."""
    global _BP
    if _BP is None:
        _BP = _binned_power_fn()
    return _BP.apply(ctx, net_load, leak_scale)


def peak_power_loss(P, beta: float):
    """Smooth peak-power loss (1/beta) * log sum_b exp(beta * P_b)."""
    import torch
    return torch.logsumexp(beta * P, dim=0) / beta


__all__ = ["Context", "GtpError", "binned_power", "peak_power_loss", "build", "load_library", "SO_PATH",
           "ABI_SYMBOLS", "fixed_point_bits", "expand_when"]
