/*
 * FP64 reference evaluator (the oracle) for the binned power waveform.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product library includes, links
 * or calls this code; only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark use it. It shares no code, header, table or constant
 * with the GPU path.
 *
 * Units: time ps (int64), slew ps, load fF, table energy fJ per transition,
 * leakage nW, supply V. Energy fJ; power mW (1 fJ/ps = 1 mW); leakage
 * energy of a rate r nW held for d ps is r*d*1e-6 fJ.
 */
#ifndef GTP_ORACLE_H
#define GTP_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  ORC_OK = 0,
  ORC_ERR_INVALID_ARG = 1,
  ORC_ERR_EVENT_ORDER = 5, /* time decreases within a gate, or a pin repeats at one time */
  ORC_ERR_EVENT_RANGE = 6, /* time outside [0, t_end) or pin > number of inputs */
  ORC_ERR_NOT_TOGGLE = 7   /* an event sets a pin to the value it already has */
};

typedef struct {
  /* cell library */
  int32_t n_cells, n_slew, n_load;
  const int32_t* n_inputs;       /* [n_cells] */
  const float* slew_axis;        /* [n_cells*n_slew] */
  const float* load_axis;        /* [n_cells*n_load] */
  const int64_t* map_base;       /* [n_cells]: entry (state s, dir d) at map_base[c] + 2*s + d */
  const int16_t* state_to_table; /* local table id of the cell */
  const int64_t* table_base;     /* [n_cells]: table k of cell c = tables[(table_base[c]+k)*n_slew*n_load ...] */
  const float* tables;           /* [table][slew i][load j] */
  const int64_t* leak_base;      /* [n_cells]: leak of state s at leak[leak_base[c] + s] */
  const float* leak;
  /* netlist */
  int64_t n_gates, n_nets;
  const int32_t* gate_cell;
  const int32_t* gate_out_net;
  const uint32_t* gate_init;     /* bit p = initial value of pin p; output pin = I */
  const float* net_load;         /* [n_nets] fF */
  const float* leak_scale;       /* [n_gates] */
  /* events: gate-major, time-sorted per gate */
  int64_t n_events;
  const int64_t* gate_off;       /* [n_gates+1] */
  const int64_t* t;
  const uint8_t* pin_bit;        /* (pin << 1) | new value */
  const float* slew;
  /* analysis parameters */
  int64_t t_end, bin_ps;
  double vdd;
  int32_t sw_mode;               /* 0: 0.5*C*V^2 per output toggle; 1: C*V^2 per output rise */
  int32_t state_all_pins;        /* 0: state index over the input pins (2^I); 1: over all pins, bit I = output (2^(I+1)) */
  int64_t glitch_clk;            /* clock period (ps) of the glitch detection; 0: no glitch analysis */
  /* state patterns (Sec. 4.1). A cell with n_tpat[c] > 0 takes its tables and
   * leakage values from patterns instead of the per-state arrays above. Table
   * pattern k of cell c is entry tpat_base[c] + k of tpat_care / tpat_value
   * (bit p = pin p; it matches a state that agrees with value on every pin
   * whose care bit is set) with tables tpat_table[2*(tpat_base[c]+k) + dir];
   * leakage pattern k is entry lpat_base[c] + k of lpat_care / lpat_value /
   * lpat_leak. A state takes its first matching pattern, scanned in order;
   * the last pattern of each list must have care = 0 (the default item, so
   * every state matches one). NULL n_tpat: no patterned cell. */
  const int32_t* n_tpat;
  const int64_t* tpat_base;
  const uint32_t* tpat_care;
  const uint32_t* tpat_value;
  const int16_t* tpat_table;
  const int32_t* n_lpat;
  const int64_t* lpat_base;
  const uint32_t* lpat_care;
  const uint32_t* lpat_value;
  const float* lpat_leak;
} orc_problem;

/* First pattern k in 0..n-1 whose care pins agree with state s (Sec. 4.1,
 * the pattern traversal that SIPL replaces), -1 when none does. */
int64_t orc_pattern_scan(int64_t n, const uint32_t* care, const uint32_t* value, uint32_t s);

/* Number of bins: ceil(t_end / bin_ps). */
int64_t orc_num_bins(const orc_problem* P);

/* Bilinear interpolation of cell c's table k at (slew, load), as used by
 * the evaluator (exported so tests can pin it on its own). */
double orc_bilerp(const orc_problem* P, int32_t c, int32_t k, double slew, double load);

/*
 * Binned energy over bins [b0, b1): E[b-b0] in fJ (P_b = E_b / bin_ps, mW).
 * leak_mode 0: leakage of every interval added bin by bin (direct);
 * leak_mode 1: fully covered bins via a difference array (same values).
 * gates: optional subset (NULL = all gates). totals (may be NULL) receives
 * [sum E_int, sum E_sw, sum E_leak, sum E_gl] over [0, t_end) for the gate
 * set, independent of the bin window (with glitch analysis on, the scaled
 * energy of a glitch event is counted in E_gl only). nthreads <= 0 uses all
 * threads. Returns ORC_* status; on error *bad_event (if not NULL) holds an
 * event.
 */
int orc_forward(const orc_problem* P, int64_t b0, int64_t b1, int leak_mode, const int64_t* gates,
                int64_t n_gate_list, double* E, double* totals, int nthreads, int64_t* bad_event);

/* Per-event state before the event's timestamp group (input pins only,
 * bit p = pin p) and bin index floor(t / bin_ps). */
int orc_event_trace(const orc_problem* P, int32_t* state_before, int64_t* bin, int64_t* bad_event);

/*
 * Gradient of a scalar loss L(P) given gP[b] = dL/dP_b for all bins:
 * grad_load[n] = dL/d(net_load[n]), grad_scale[g] = dL/d(leak_scale[g]).
 * leak_mode as in orc_forward (0: bin by bin; 1: cumulative integral).
 */
int orc_adjoint(const orc_problem* P, const double* gP, int leak_mode, double* grad_load, double* grad_scale,
                int nthreads);

/*
 * Per-gate report: gate_e[4*g + k] = energy (fJ) of gate g over [0, t_end),
 * k = 0 leakage, 1 internal, 2 switching, 3 glitch; *t_max = the latest event
 * time (the horizon of the paper's average power p = E / t_max), -1 without
 * events.
 */
int orc_gate_report(const orc_problem* P, double* gate_e, int64_t* t_max, int nthreads);

/* Validation only: first offending event in gate-major order. */
int orc_validate(const orc_problem* P, int64_t* bad_event);

/* Threads the evaluator would use for nthreads <= 0. */
int orc_max_threads(void);

#ifdef __cplusplus
}
#endif
#endif
