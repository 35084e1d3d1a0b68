/*
 * gtpower — C ABI of the MI355X (gfx950) binned power-waveform library.
 *
 * The library turns per-gate toggle-event streams into a time-binned power
 * waveform (the power models of the paper's Sec. 2.2 evaluated in time as in
 * Sec. 2.4, fused as in Sec. 4.3 / Algorithm 1): every event gets a
 * state-indexed internal energy lookup (Sec. 4.1: the gate's input state
 * selects a table, which is interpolated bilinearly over input slew x output
 * load, Sec. 2.2), output toggles add switching energy (Eq. switching energy;
 * see gtp_params), the leakage of each held input state is charged for its
 * duration (Eq. leakage energy) and everything is accumulated into
 * fixed-width time bins, an interval being split over the bins it overlaps
 * (Sec. 2.4).
 * The adjoint gives d(loss)/d(net load) and d(loss)/d(per-gate leakage
 * scale) for a loss of the binned power.
 *
 * Units: time ps (int64), slew ps, load fF, table energy fJ per transition,
 * leakage nW, supply V; power mW (1 fJ/ps = 1 mW).
 *
 * Conventions for every call:
 *   - Status returns only; nothing aborts and no C++ exception leaves the ABI.
 *     gtp_last_error() gives a message for the last non-OK status of a ctx.
 *   - Device work is asynchronous on the ctx stream (a hipStream_t passed as
 *     void*; NULL = the null stream). A non-OK status reports argument or
 *     enqueue errors; conditions found by kernels (a leakage scale out of
 *     range, an invalid event when validating) are reported by the next
 *     synchronising call: gtp_sync(), gtp_load_events(validate=1).
 *   - "DEVICE" pointers are HIP device memory on the ctx device; "HOST"
 *     pointers are host memory. Library and netlist arrays are copied into
 *     ctx-owned memory; event arrays are BORROWED (they are large) and must
 *     stay alive and unchanged until the next gtp_load_events or gtp_destroy.
 *     Outputs are caller-allocated and overwritten.
 *   - A ctx is not thread-safe; use one per host thread.
 */
#ifndef GTPOWER_H
#define GTPOWER_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gtp_ctx_s* gtp_ctx;

typedef enum {
  GTP_OK = 0,
  GTP_ERR_INVALID_ARG = 1,   /* null pointer, negative or mismatched size, bad table */
  GTP_ERR_OUT_OF_MEMORY = 2, /* device allocation failed */
  GTP_ERR_HIP = 3,           /* a HIP runtime call failed */
  GTP_ERR_NOT_LOADED = 4,    /* library, netlist, events or params missing */
  GTP_ERR_EVENT_ORDER = 5,   /* time decreases within a gate, or a pin repeats at one time */
  GTP_ERR_EVENT_RANGE = 6,   /* time outside [0, t_end) or pin above the output pin */
  GTP_ERR_NOT_TOGGLE = 7,    /* an event sets a pin to the value it already holds */
  GTP_ERR_UNSUPPORTED = 8,   /* valid input outside the sizes this build handles */
  GTP_ERR_SCALE_RANGE = 9,   /* a leakage scale is negative, not finite or above GTP_MAX_LEAK_SCALE */
  GTP_ERR_LOAD_RANGE = 10    /* a net load is negative, not finite or above 4x the library's largest load knot */
} gtp_status;

/* Leakage scales must lie in [0, GTP_MAX_LEAK_SCALE]; the fixed-point range of
 * the leakage accumulators is sized from it and the library's largest value. */
#define GTP_MAX_LEAK_SCALE 16.0f

/* Create a context on HIP device `hip_device`, enqueuing on `hip_stream`. */
gtp_status gtp_create(gtp_ctx* out, int hip_device, void* hip_stream);
/* Free every ctx-owned buffer (synchronises the stream first). NULL is a no-op. */
gtp_status gtp_destroy(gtp_ctx ctx);
/* Change the stream later calls enqueue on. */
gtp_status gtp_set_stream(gtp_ctx ctx, void* hip_stream);
/* Message for the last non-OK status on ctx (never NULL; "" if none). */
const char* gtp_last_error(gtp_ctx ctx);
/* Wait for the ctx stream; report a condition flagged by kernels since the
 * last check (GTP_ERR_LOAD_RANGE, GTP_ERR_SCALE_RANGE) or a HIP error. */
gtp_status gtp_sync(gtp_ctx ctx);

/*
 * Fixed-point range of the bin accumulators (host only, no device work).
 * Bin energies are accumulated as exact integers in units of 2^-m fJ (the
 * leakage rate in units of 1e6 * 2^-m nW, so a rate unit held for 1 ps is one
 * energy unit); m is chosen per event set and bin width as the largest
 * m <= 40 with
 *   2^m * (max_bin_events * event_energy_fj + bin_ps * leak_rate_fj_per_ps) < 2^62
 *   2^m * 1e-6 * leak_value_nw < 2^30   (a quantised rate fits 30 bits)
 * where event_energy_fj bounds |energy| of one event, leak_rate_fj_per_ps the
 * total leakage rate and leak_value_nw one gate's scaled leakage value. With
 * that m no bin and no rate can wrap. Returns GTP_ERR_UNSUPPORTED when m would
 * fall below 30 (the quantised leakage rates would then miss the 1e-5
 * relative budget of the waveform, whose readings are Sec. 2.4's overlap rule
 * and Eq. leakage energy), GTP_ERR_INVALID_ARG for negative or non-finite
 * inputs. gtp_forward applies it with bounds taken from the library (largest
 * table entry, slew and load extrapolation factors), the netlist (the sum of
 * every gate's largest leakage value at the largest scale) and the packed
 * events (most events in one bin).
 */
typedef struct {
  int64_t max_bin_events;
  int64_t bin_ps;
  double event_energy_fj;
  double leak_rate_fj_per_ps;
  double leak_value_nw;
} gtp_range;
gtp_status gtp_fixed_point_bits(const gtp_range* r, int32_t* m);

/*
 * Expansion of state patterns with don't-care pins into a per-state array
 * (host only, no device work, no context): Sec. 4.1, SIPL, where a pattern
 * that fixes only some pins applies to every state that agrees with it on
 * those pins, filled by enumerating the assignments of its don't-care pins.
 * Pattern k matches state s when (s & care[k]) == (value[k] & care[k]) (bit p
 * = pin p); out[s] = item[k] of the first pattern in array order that matches
 * s, default_item when none does (the paper assumes patterns that do not
 * overlap; first-match is the reading for those that do).
 *   n_pins      pins of the state index, 0..16 (the direct-array limit
 *               the paper uses); out has 2^n_pins entries (HOST, written)
 *   care, value, item   n_patterns >= 0 entries each (HOST, read)
 * Errors: GTP_ERR_INVALID_ARG for n_pins outside 0..16, a null array, or a
 * care bit at or above n_pins (out is then unspecified).
 */
gtp_status gtp_expand_when(int32_t n_pins, int32_t n_patterns, const uint32_t* care, const uint32_t* value,
                           const int32_t* item, int32_t default_item, int32_t* out);

/*
 * Cell library (HOST pointers, copied). For cell c with I = n_inputs[c]
 * input pins (pins 0..I-1; the output is pin I):
 *   state s = sum_p value(p) * 2^p over the input pins (Sec. 4.1, the
 *   state-indexed lookup: bit p = input pin p), or, with all_pin_state = 1,
 *   over every pin of the cell (bit I = the output; 2^(I+1) states, Sec. 4.1
 *   indexes the array by all of the cell's pins);
 *   state_to_table[map_base[c] + 2*s + dir] = local table id k of the cell
 *   for an event with new value dir (1 = rise) at input state s;
 *   table k: tables_fj[((table_base[c] + k) * n_slew + i) * n_load + j] = energy
 *   at slew_axis_ps[c*n_slew + i], load_axis_ff[c*n_load + j];
 *   leak_nw[leak_base[c] + s] = leakage power at state s.
 * Axes strictly increasing; n_slew, n_load in [2, 16]; leakage values
 * finite and >= 0; every table id in range. Local table ids may be shared by
 * several (state, dir) pairs. A cell given by these per-state arrays has at
 * most 8 state pins (I in [1, 8], I + 1 <= 8 with all_pin_state).
 *
 * State patterns (Sec. 4.1, optional: n_tpat NULL means none). A cell c with
 * n_tpat[c] > 0 is given by Liberty-style `when` patterns instead (its
 * map_base and leak_base entries are then ignored), with I in [1, 31] (the
 * I + 1 pin values fit 32 bits):
 *   table pattern k (0 <= k < n_tpat[c]) is entry i = tpat_base[c] + k of
 *   tpat_care / tpat_value (bit p = pin p of the state index) and selects
 *   local tables tpat_table[2*i + dir]; it matches state s when
 *   (s & care) == (value & care) (pins outside care are don't-cares);
 *   leakage pattern k (0 <= k < n_lpat[c]) is entry i = lpat_base[c] + k of
 *   lpat_care / lpat_value with value lpat_leak_nw[i].
 * A state takes the first matching pattern of each list. Each list holds 1 to
 * 256 patterns and its last pattern has care = 0 (the cell's default, the
 * Liberty group without a `when`), so every state matches. Care bits lie
 * below the cell's state-pin count. The library expands the patterns of a
 * cell with at most 16 state pins into per-state arrays (the expansion of
 * gtp_expand_when; on chip for at most 8 state pins, in device memory above)
 * and scans the patterns of wider cells in order at every lookup (the
 * fallback of Sec. 4.1 for cells with more than 16 pins). Either way the
 * result equals the first-match scan.
 */
typedef struct {
  int32_t n_cells, n_slew, n_load;
  const int32_t* n_inputs;      /* [n_cells] */
  const float* slew_axis_ps;    /* [n_cells * n_slew] */
  const float* load_axis_ff;    /* [n_cells * n_load] */
  const int64_t* map_base;      /* [n_cells] */
  const int16_t* state_to_table;
  const int64_t* table_base;    /* [n_cells] */
  const float* tables_fj;
  const int64_t* leak_base;     /* [n_cells] */
  const float* leak_nw;
  int64_t n_map, n_tables, n_leak; /* lengths of state_to_table, tables (in tables), leak_nw */
  int32_t all_pin_state;           /* 0: state over the input pins; 1: over every pin (output = bit I) */
  const int32_t* n_tpat;           /* [n_cells] or NULL: table patterns per cell (0: per-state arrays) */
  const int64_t* tpat_base;        /* [n_cells] */
  const uint32_t* tpat_care;       /* [n_tpat_total] */
  const uint32_t* tpat_value;      /* [n_tpat_total] */
  const int16_t* tpat_table;       /* [2 * n_tpat_total]: local table id (fall, rise) */
  const int32_t* n_lpat;           /* [n_cells] leakage patterns per cell */
  const int64_t* lpat_base;        /* [n_cells] */
  const uint32_t* lpat_care;       /* [n_lpat_total] */
  const uint32_t* lpat_value;      /* [n_lpat_total] */
  const float* lpat_leak_nw;       /* [n_lpat_total] */
  int64_t n_tpat_total, n_lpat_total;
} gtp_library;
gtp_status gtp_load_library(gtp_ctx ctx, const gtp_library* lib);

/*
 * Netlist (DEVICE pointers, copied): gate g is an instance of cell
 * gate_cell[g] driving net gate_out_net[g]; bit p of gate_init_bits[g] is the
 * initial value of pin p (inputs 0..I-1, output I), i.e. the gate state of
 * Sec. 2.1 (the vector of the values on all pins of a gate) at time 0; the
 * switching energy of Eq. switching energy charges the load of the output
 * net. Requires a library. Errors: INVALID_ARG for a cell or net index out of
 * range (checked on the device, synchronises) or a null array, NOT_LOADED
 * without a library. Any failure leaves the ctx with no netlist and no events
 * (the previous ones are dropped).
 */
gtp_status gtp_load_netlist(gtp_ctx ctx, int64_t n_gates, int64_t n_nets, const int32_t* gate_cell,
                            const int32_t* gate_out_net, const uint32_t* gate_init_bits);

/*
 * Toggle events (DEVICE pointers, BORROWED), gate-major: the events of gate g
 * are [gate_off[g], gate_off[g+1]), sorted by time (events of one gate that
 * share a time form a group and may come in any order within it).
 * pin_bit = (pin << 1) | new_value; every event toggles its pin: the
 * value-timestamp pairs of Sec. 2.1, merged over the pins of a gate (the
 * per-gate activity the framework of Sec. 5 hands to the GPU).
 * Window [0, t_end); every t in it. Arrays 16-byte aligned.
 */
typedef struct {
  int64_t n_events, t_end_ps;
  const int64_t* gate_off;  /* [n_gates + 1], gate_off[0] = 0, gate_off[n_gates] = n_events */
  const int64_t* t_ps;      /* [n_events] */
  const uint8_t* pin_bit;   /* [n_events] */
  const float* slew_ps;     /* [n_events] */
} gtp_events;
/* Record the events and (re)build the execution plan. validate = 1 also
 * checks every event on the device and synchronises: the first offending
 * event in gate-major order gives GTP_ERR_EVENT_ORDER / _EVENT_RANGE /
 * _NOT_TOGGLE (its index in gtp_last_error). validate = 0 trusts the input
 * (invalid events then give unspecified waveforms, never a fault). */
gtp_status gtp_load_events(gtp_ctx ctx, const gtp_events* ev, int validate);
/* Index of the event named by the last validation failure, else -1. */
int64_t gtp_bad_event(gtp_ctx ctx);

/*
 * Analysis parameters. Bins are half-open [b*bin_ps, (b+1)*bin_ps),
 * n_bins = ceil(t_end / bin_ps); a partial last bin is still divided by
 * bin_ps. sw_mode 0: switching energy 0.5*C*V^2 on every output toggle;
 * sw_mode 1: C*V^2 on an output rise only (the paper's Eq. switching energy).
 * bin_ps in [1, 2^22].
 * glitch_clk_ps > 0 turns on the clock-cycle glitch detection (Sec. 2.4,
 * Sec. 4.3): an event that is not its pin's first in its clock cycle
 * [k*glitch_clk_ps, (k+1)*glitch_clk_ps) is a glitch event; its internal plus
 * switching energy is scaled by r = min(1, (2*pw / (rSlew + fSlew))^2) (Eq.
 * glitch scaling ratio; pw = time since the pin's previous event, the slews
 * those of that event and this one) and counted as glitch energy. The
 * waveform then carries the scaled energy. 0 = off.
 */
typedef struct {
  double vdd;
  int64_t bin_ps;
  int64_t glitch_clk_ps;
  int32_t sw_mode;
} gtp_params;
gtp_status gtp_set_params(gtp_ctx ctx, const gtp_params* p);
gtp_status gtp_num_bins(gtp_ctx ctx, int64_t* n_bins);

/*
 * Execution choices. algo 0: packed tile-major path (the default: events
 * regrouped once into time tiles, one workgroup per tile, bins accumulated in
 * LDS); algo 1: one gate per thread with global atomics (baseline).
 * bins_per_tile_log2: 0 = automatic, else 2..13 (bins per time tile of the
 * packed path; the tile's bins and the library image must fit in 160 KB of
 * LDS). tile_threads: threads per time-tile workgroup of the packed path,
 * 0 = automatic, else 256, 512 or 1024. unit_events: longest run of one
 * gate's events one lane takes (the density split: denser gates are cut into
 * more runs), 0 = 8, else 1..16. gate_block_log2: gates per sort block of the
 * packed layout (log2), 0 = 13, else 6..20 (the packed adjoint holds 16 bytes
 * per gate of a block in LDS; when they do not fit it runs the gate-major
 * walk). Both paths give bit-identical waveforms.
 */
typedef struct {
  int32_t algo;
  int32_t bins_per_tile_log2;
  int32_t tile_threads;
  int32_t unit_events;
  int32_t gate_block_log2;
} gtp_tuning;
gtp_status gtp_set_tuning(gtp_ctx ctx, const gtp_tuning* t);
gtp_status gtp_get_tuning(gtp_ctx ctx, gtp_tuning* t);

/*
 * Statistics of the packed layout (builds it if needed, which synchronises):
 * events packed (those with times in the window), units (runs of at most 16
 * events of one gate in one time tile), wavefront groups of 64 units, time
 * tiles, bins per tile (log2), the largest group count of one tile, device
 * bytes of the packed arrays, the time the last build took (ms) and the lane
 * steps (sum over groups of the longest unit: a wavefront spends that many
 * event steps on a group, so n_events_packed / (64 * lane_steps) is the
 * fraction of busy lanes).
 */
typedef struct {
  int64_t n_events_packed, n_units, n_groups;
  int32_t n_tiles, tile_log2, max_tile_groups;
  int64_t packed_bytes;
  double pack_ms;
  int64_t lane_steps;
} gtp_plan_stats;
gtp_status gtp_plan_info(gtp_ctx ctx, gtp_plan_stats* out);

/*
 * Autotuner (the paper tunes its partition parameters per workload, Sec. 4.2
 * and Sec. 6.5): times the packed forward on the loaded events (and, if a
 * batch is loaded, the batched forward) for candidate tunings (bins per tile,
 * threads per tile workgroup, longest run per lane, gate-block size), keeps
 * the fastest and applies it with gtp_set_tuning. cache_json_path (HOST
 * string, may be NULL): a JSON file of earlier choices keyed by device and
 * workload signature; a hit skips the timing, a miss appends the choice.
 * Synchronises; rebuilds the packed layouts.
 */
gtp_status gtp_autotune(gtp_ctx ctx, const char* cache_json_path);

/*
 * Forward: power_mw[b] (DEVICE, [n_bins], FP32) = binned power for net loads
 * net_load_ff (DEVICE, [n_nets]) and leakage scales leak_scale (DEVICE,
 * [n_gates]; NULL = all 1). Per event the internal energy of the table the
 * state before the event's timestamp group selects (Sec. 4.1), interpolated
 * at (slew, load) (Sec. 2.2), plus switching energy on output events (Eq.
 * switching energy, see sw_mode); leakage of every held state for its
 * duration split over the bins it overlaps (Sec. 2.4, Eq. leakage energy);
 * the per-timestamp order of Algorithm 1 (look up every event of a group with
 * the state before it, then apply the group). Accumulation is exact int64
 * fixed point (gtp_fixed_point_bits), so the result does not depend on the
 * execution order. Loads must lie in [0, 4 x the largest load knot], scales
 * in [0, GTP_MAX_LEAK_SCALE] (else GTP_ERR_LOAD_RANGE / _SCALE_RANGE at the
 * next gtp_sync, the value used as 0). The first call after new events or
 * parameters builds the packed layout (synchronises; gtp_plan_info reports
 * its time); power_mw must hold n_bins floats.
 */
gtp_status gtp_forward(gtp_ctx ctx, const float* net_load_ff, const float* leak_scale, float* power_mw);

/*
 * Allocation-free forward, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same result as gtp_forward (bit for bit, same kernels), but
 * its per-call buffers (gate records, bins, tile sums: 8*n_gates +
 * 16*n_bins + 16*n_tiles + 8*ceil(n_gates/256) bytes, each part rounded up to
 * 256) live in a fixed 64 MiB device array of the library, one per GPU, so the
 * call makes no hipMalloc, hipFree or allocating library call. Requirements:
 * the packed layout already built for the loaded events and parameters (by
 * gtp_plan_info or an earlier gtp_forward: GTP_ERR_NOT_LOADED otherwise),
 * algo 0, and buffers that fit the array (GTP_ERR_UNSUPPORTED otherwise; the
 * 1M-gate, 2M-bin workload needs about 40 MB). Every call on a GPU shares
 * that GPU's array: calls that overlap on one GPU (any contexts, any streams)
 * race and must be serialised by the caller. Profiling records are not made
 * for this call.
 */
gtp_status gtp_forward_noalloc(gtp_ctx ctx, const float* net_load_ff, const float* leak_scale, float* power_mw);

/*
 * Adjoint (no counterpart in the paper: the gradient of a loss of the
 * forward's waveform, through the interpolation of Sec. 2.2, Eq. switching
 * energy and Eq. leakage energy): given grad_power[b] = dL/dP_b (DEVICE,
 * [n_bins]) writes
 * grad_net_load[n] = dL/d(net_load_ff[n]) (DEVICE, [n_nets]; nets no gate
 * drives get 0) and grad_leak_scale[g] = dL/d(leak_scale[g]) (DEVICE,
 * [n_gates]). Event times and states are not differentiated.
 */
gtp_status gtp_adjoint(gtp_ctx ctx, const float* net_load_ff, const float* leak_scale, const float* grad_power,
                       float* grad_net_load, float* grad_leak_scale);

/*
 * Batched traces: n_traces stimulus traces over the loaded netlist, each a
 * gtp_events struct of DEVICE pointers, BORROWED as in gtp_load_events (trace
 * i covers its own window [0, t_end_i)). Requires gtp_set_params (the traces share the
 * bin width and switching mode) and replaces any earlier batch. validate = 1
 * checks every event as gtp_load_events does and synchronises; a failure
 * names the trace in gtp_last_error, and gtp_bad_event gives the event index
 * within that trace. The packed layouts are built on the first batched call.
 */
gtp_status gtp_load_traces(gtp_ctx ctx, int32_t n_traces, const gtp_events* traces, int validate);

/* Total bins of the loaded batch; offsets (HOST, [n_traces + 1], may be NULL)
 * gets the first bin of every trace in the concatenated output. */
gtp_status gtp_batch_bins(gtp_ctx ctx, int64_t* total, int64_t* offsets);

/*
 * Forward of every trace of the batch in one persistent launch (the chunk
 * loop of Sec. 5 processes event chunks one after another with the same
 * kernel; here all traces share one launch): workgroups take (trace, time
 * tile) work items from a device queue, largest first, so uneven trace
 * lengths balance. The traces share one fixed-point exponent (the smallest
 * any trace needs). power_mw (DEVICE, [total bins]) gets the
 * waveforms back to back (trace i from offsets[i]). use_graph = 1 records the
 * whole call (gate parameters, queue reset, persistent kernel, leakage scan,
 * finalize) as a HIP graph on its first use and replays it afterwards; it is
 * recorded again when net_load_ff, leak_scale or power_mw differ from the
 * recorded pointers or the batch, parameters or tuning change.
 */
gtp_status gtp_forward_batched(gtp_ctx ctx, const float* net_load_ff, const float* leak_scale, float* power_mw,
                               int use_graph);

/* Forward of trace `trace` of the batch alone (its own launches), into
 * power_mw (DEVICE, [its bins]): the per-trace reference of the batched call. */
gtp_status gtp_forward_trace(gtp_ctx ctx, int32_t trace, const float* net_load_ff, const float* leak_scale,
                             float* power_mw);

/*
 * Per-gate power report (Sec. 4.4 reduces per-gate leakage, internal,
 * switching and glitch power; Sec. 5 reports them per gate and for the
 * design, with the waveform's peak): for the loaded events and parameters,
 *   gate_energy_fj (DEVICE, [n_gates * 4], FP64): gate g's energy over the
 *     window [0, t_end) as (leakage, internal, switching, glitch) at
 *     [4*g .. 4*g+3]; a glitch event's scaled energy counts as glitch only;
 *   totals (HOST, [12]): [0..3] the design sums of the four components (fJ),
 *     [4] t_max = the latest event time (ps; -1 without events), [5] the
 *     largest value of power_mw (mW; NaN if power_mw is NULL), [6..9] the
 *     paper's average powers p = E / t_max of the four components (Eq.
 *     average power; mW, NaN when t_max <= 0), [10] the average total power
 *     over the window (sum of the components / t_end, mW), [11] t_end (ps).
 * power_mw (DEVICE, [n_bins], may be NULL): a waveform from gtp_forward, for
 * the peak. Energies are the FP32 per-event values the forward uses, summed
 * in FP64 per gate. Synchronises.
 */
gtp_status gtp_gate_report(gtp_ctx ctx, const float* net_load_ff, const float* leak_scale, const float* power_mw,
                           double* gate_energy_fj, double* totals);

/*
 * Streamed evaluation of one trace larger than device memory (Sec. 5: the
 * events are split into chunks that fit the GPU, and the next chunk is made
 * ready while the GPU works on the current one). The trace [0, t_end) is cut
 * at times 0 = t_0 < t_1 < ... < t_K = t_end; window k holds every event with
 * t_k <= t < t_{k+1}, as a gate-major CSR over all gates of the netlist with
 * absolute times (the layout of gtp_load_events; its t_end_ps is not used).
 * Each cut is a multiple of bin_ps, and of glitch_clk_ps when glitch
 * detection is on, so every bin and every clock cycle lies inside one window.
 * The library carries every gate's pin values from one window into the next,
 * so the result is the waveform of the whole trace (each window's bins are
 * evaluated with the fixed-point exponent its own events allow).
 *
 *   gtp_stream_begin  opens a stream of t_end_ps (library, netlist and
 *       parameters loaded; the loaded events are dropped). validate = 1
 *       checks every window's events as gtp_load_events does (an error ends
 *       the stream). While a stream is open every other call on ctx returns
 *       GTP_ERR_INVALID_ARG.
 *   gtp_stream_push   enqueues the copy of the next window's HOST arrays
 *       (pinned memory lets the copy overlap the GPU work) into one of two
 *       device staging slots, on a copy stream of the library; at most two
 *       windows are pending. Waits only for the window that last used the
 *       slot. The host arrays must stay unchanged until the gtp_stream_step
 *       that evaluates the window returns.
 *   gtp_stream_step   evaluates the oldest pending window and writes its bins
 *       [t_k / bin_ps, ceil(t_{k+1} / bin_ps)) of power_mw (DEVICE,
 *       ceil(t_end / bin_ps) floats for the whole trace); net_load_ff and
 *       leak_scale as in gtp_forward. The copy of a window pushed before the
 *       step overlaps it.
 *   gtp_stream_end    closes the stream (pending windows are dropped) and
 *       restores the netlist's initial pin values.
 * Errors: GTP_ERR_INVALID_ARG for cuts out of order or off the bin (clock)
 * grid, a third pending window, a window gate_off that does not run from 0
 * to its n_events; GTP_ERR_NOT_LOADED without an open stream.
 */
gtp_status gtp_stream_begin(gtp_ctx ctx, int64_t t_end_ps, int32_t validate);
gtp_status gtp_stream_push(gtp_ctx ctx, const gtp_events* window_host, int64_t t0_ps, int64_t t1_ps);
gtp_status gtp_stream_step(gtp_ctx ctx, const float* net_load_ff, const float* leak_scale, float* power_mw);
gtp_status gtp_stream_end(gtp_ctx ctx);

/*
 * Per-event trace of the state tracking (DEVICE outputs, [n_events]):
 * state_before[e] = input state of e's gate before e's timestamp group
 * (the state every event of the group is looked up with, Algorithm 1),
 * bin[e] = floor(t_e / bin_ps).
 */
gtp_status gtp_debug_event_trace(gtp_ctx ctx, int32_t* state_before, int64_t* bin);

/*
 * Kernel timing. gtp_profile_enable(ctx, 1) clears earlier records and makes
 * every later launch of the ctx record a HIP event pair on the ctx stream
 * around it (0 stops recording). gtp_profile_read synchronises the stream and
 * writes, for up to cap kernels in first-launch order, the kernel name (owned
 * by ctx, valid until the next gtp_profile_enable or gtp_destroy), its number
 * of launches and their summed duration in ms; *n_out = number of kernels.
 */
gtp_status gtp_profile_enable(gtp_ctx ctx, int enable);
gtp_status gtp_profile_read(gtp_ctx ctx, int32_t cap, const char** names, int64_t* launches, double* total_ms,
                            int32_t* n_out);

/* Bytes of ctx-owned device memory currently allocated. */
int64_t gtp_device_bytes(gtp_ctx ctx);

#ifdef __cplusplus
}
#endif
#endif
