/*
 * FP64 reference evaluator (the oracle) for the time-binned power waveform.
 *
 * TEST INFRASTRUCTURE ONLY: used by tests, the smoke check and the CPU
 * baseline of the benchmark; never by the product library, with which it
 * shares no code.
 *
 * What it computes (paper Sec. 2.2 power models, Sec. 2.4 Naive-D/Naive-L,
 * Sec. 4.3 fused kernel, Algorithm 1). For each gate, in time order, one
 * timestamp group at a time (all events of the gate that share a time):
 *   1. leakage of the interval since the previous group at the leakage value
 *      selected by the current input state (state-indexed lookup, Sec. 4.1),
 *      E_leak = p_leak * dt (Eq. leakage energy), split over the time bins it
 *      overlaps in proportion to the overlap (Sec. 2.4, Naive-L);
 *   2. for every event of the group, the internal energy read from the table
 *      chosen by the state before the group and the event's new value, by
 *      bilinear interpolation at (input slew, output load) (Sec. 2.2), plus
 *      switching energy for an output toggle, added to the bin holding the
 *      event's time (Sec. 4.3, dynamic power);
 *   3. the group's events are applied to the gate state.
 * After the last group the leakage runs to the end of the window.
 *
 * Glitch power (optional, glitch_clk > 0; Sec. 2.2 Glitch Power, the
 * clock-cycle detection of Sec. 2.4 and Sec. 4.3 GlitchDetectUpdate, Eq.
 * glitch scaling ratio): per pin, a counter of the pin's events in the
 * current clock cycle (reset when the pin's cycle changes). An event that is
 * not its pin's first in the cycle is a glitch event: its dynamic energy
 * (internal + switching) is scaled by r = min(1, (2 pw / (rSlew + fSlew))^2),
 * pw = time since the pin's previous event, rSlew + fSlew = the slews of that
 * event and this one (a rise and a fall: the pin toggles), and is counted as
 * glitch energy (the waveform gets the scaled energy, the internal and
 * switching totals nothing).
 *
 * Readings where the paper is silent (also listed in the design doc):
 *   - switching energy: 0.5*C*V^2 on every output toggle (sw_mode 0), or the
 *     paper's C*V^2 on an output rise only (sw_mode 1, Eq. switching energy);
 *   - state index over the input pins, bit p = value of input pin p
 *     (state_all_pins = 1: over all pins, bit I = the output, the SIPL index of
 *     Sec. 4.1 over every pin of the cell);
 *   - table direction = the event's own new value (1 = rise);
 *   - bins are half-open [b*D, (b+1)*D); a partial last bin is still divided
 *     by D; events must lie in [0, t_end);
 *   - interpolation extrapolates linearly outside the axes; a value on a knot
 *     uses the segment starting at that knot (the last knot: last segment);
 *   - per-gate leakage scale lambda multiplies every leakage value.
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC oracle.c -o liboracle.so -lm
 * A -DORC_PLANT=n build plants deliberate mistakes for the tests that check
 * the pins catch them; a normal build has none.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef ORC_PLANT
#define ORC_PLANT 0
#endif

int orc_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

int64_t orc_num_bins(const orc_problem* P) { return (P->t_end + P->bin_ps - 1) / P->bin_ps; }

/* index of the axis segment used for x: the segment [a_i, a_{i+1}] with
 * i = clamp(first knot > x, minus one, to [0, n-2]) */
static int seg_index(const float* axis, int n, double x) {
  int ub = 0;
  while (ub < n && (double)axis[ub] <= x) ++ub; /* first knot strictly above x */
  int i = ub - 1;
  if (i < 0) i = 0;
  if (i > n - 2) i = n - 2;
  return i;
}

static const float* table_ptr(const orc_problem* P, int32_t c, int32_t k) {
  return P->tables + (P->table_base[c] + k) * (int64_t)P->n_slew * P->n_load;
}

static double tab(const orc_problem* P, const float* T, int i, int j) {
#if ORC_PLANT == 2
  /* planted: transposed operand */
  return (double)T[j * P->n_slew + i];
#else
  return (double)T[i * P->n_load + j];
#endif
}

double orc_bilerp(const orc_problem* P, int32_t c, int32_t k, double slew, double load) {
  const float* sa = P->slew_axis + (int64_t)c * P->n_slew;
  const float* la = P->load_axis + (int64_t)c * P->n_load;
  int i = seg_index(sa, P->n_slew, slew);
  int j = seg_index(la, P->n_load, load);
  double a = (slew - sa[i]) / ((double)sa[i + 1] - sa[i]);
  double b = (load - la[j]) / ((double)la[j + 1] - la[j]);
  const float* T = table_ptr(P, c, k);
  return (1 - a) * (1 - b) * tab(P, T, i, j) + a * (1 - b) * tab(P, T, i + 1, j) +
         (1 - a) * b * tab(P, T, i, j + 1) + a * b * tab(P, T, i + 1, j + 1);
}

/* d(bilerp)/d(load) on the segment the forward evaluation uses */
static double bilerp_dload(const orc_problem* P, int32_t c, int32_t k, double slew, double load) {
  const float* sa = P->slew_axis + (int64_t)c * P->n_slew;
  const float* la = P->load_axis + (int64_t)c * P->n_load;
  int i = seg_index(sa, P->n_slew, slew);
  int j = seg_index(la, P->n_load, load);
  double a = (slew - sa[i]) / ((double)sa[i + 1] - sa[i]);
  const float* T = table_ptr(P, c, k);
  double d0 = tab(P, T, i, j + 1) - tab(P, T, i, j);
  double d1 = tab(P, T, i + 1, j + 1) - tab(P, T, i + 1, j);
  return ((1 - a) * d0 + a * d1) / ((double)la[j + 1] - la[j]);
}

/* switching energy of an output event with new value v (Eq. switching energy) */
static double sw_energy(const orc_problem* P, double C, int v) {
  double V2 = P->vdd * P->vdd;
  if (P->sw_mode == 1) return v ? C * V2 : 0.0;
#if ORC_PLANT == 3
  return C * V2; /* planted: dropped factor 1/2 */
#else
  return 0.5 * C * V2;
#endif
}

static double sw_energy_dC(const orc_problem* P, int v) {
  double V2 = P->vdd * P->vdd;
  if (P->sw_mode == 1) return v ? V2 : 0.0;
#if ORC_PLANT == 9
  return 0.0; /* planted: dropped switching term in the gradient */
#else
  return 0.5 * V2;
#endif
}

/* mask of the n low bits, n in 0..32 */
static uint32_t low_bits(int n) { return n >= 32 ? 0xffffffffu : (1u << n) - 1u; }

int64_t orc_pattern_scan(int64_t n, const uint32_t* care, const uint32_t* value, uint32_t s) {
  for (int64_t k = 0; k < n; ++k) {
#if ORC_PLANT == 14
    if ((s & care[k]) == value[k]) return k; /* planted: value bits outside care compared too */
#else
    if ((s & care[k]) == (value[k] & care[k])) return k;
#endif
  }
  return -1;
}

static int patterned(const orc_problem* P, int32_t c) { return P->n_tpat && P->n_tpat[c] > 0; }

/* local table id of cell c for state s and new value dir: the per-state
 * array, or the first matching table pattern */
static int32_t table_id(const orc_problem* P, int32_t c, uint32_t s, int dir) {
  if (!patterned(P, c)) return P->state_to_table[P->map_base[c] + 2 * (int64_t)s + dir];
  const int64_t b = P->tpat_base[c];
  const int64_t k = orc_pattern_scan(P->n_tpat[c], P->tpat_care + b, P->tpat_value + b, s);
  return P->tpat_table[2 * (b + k) + dir];
}

/* leakage value (nW) of cell c at state s */
static double leak_value(const orc_problem* P, int32_t c, uint32_t s) {
  if (!patterned(P, c)) return (double)P->leak[P->leak_base[c] + s];
  const int64_t b = P->lpat_base[c];
  const int64_t k = orc_pattern_scan(P->n_lpat[c], P->lpat_care + b, P->lpat_value + b, s);
  return (double)P->lpat_leak[b + k];
}

/* every pattern list non-empty and ending in a care = 0 pattern */
static int check_patterns(const orc_problem* P) {
  if (!P->n_tpat) return ORC_OK;
  for (int32_t c = 0; c < P->n_cells; ++c) {
    if (!patterned(P, c)) continue;
    if (!P->n_lpat || P->n_lpat[c] < 1) return ORC_ERR_INVALID_ARG;
    if (P->tpat_care[P->tpat_base[c] + P->n_tpat[c] - 1] != 0u) return ORC_ERR_INVALID_ARG;
    if (P->lpat_care[P->lpat_base[c] + P->n_lpat[c] - 1] != 0u) return ORC_ERR_INVALID_ARG;
  }
  return ORC_OK;
}

static int64_t bin_of(const orc_problem* P, int64_t t) {
#if ORC_PLANT == 5
  return (t + P->bin_ps / 2) / P->bin_ps; /* planted: rounds instead of floor */
#else
  return t / P->bin_ps;
#endif
}

/* Bin accumulator for one thread: direct adds or difference array. */
typedef struct {
  int64_t b0, b1;
  double* E;    /* [b1-b0] */
  double* diff; /* [b1-b0+1], leak_mode 1 */
  int mode;
} acc_t;

static void acc_add(acc_t* A, int64_t b, double v) {
  if (b >= A->b0 && b < A->b1) A->E[b - A->b0] += v;
}

/* leakage at rate r (nW) over [t0, t1), split over bins by overlap */
static void add_leak(const orc_problem* P, acc_t* A, int64_t t0, int64_t t1, double r) {
  if (t1 <= t0) return;
  const int64_t D = P->bin_ps;
  const double k = r * 1e-6; /* fJ per ps */
  if (A->mode == 0) {
    int64_t bl = t0 / D, bh = (t1 - 1) / D;
    if (bl < A->b0) bl = A->b0;
    if (bh > A->b1 - 1) bh = A->b1 - 1;
    for (int64_t b = bl; b <= bh; ++b) {
      int64_t lo = b * D > t0 ? b * D : t0;
      int64_t hi = (b + 1) * D < t1 ? (b + 1) * D : t1;
      if (hi > lo) A->E[b - A->b0] += k * (double)(hi - lo);
    }
    return;
  }
  /* partial bins at both ends, whole bins [bf, bl) by a difference array */
  int64_t bt0 = t0 / D, bt1 = t1 / D;
  if (bt0 == bt1 || (bt0 + 1 == bt1 && t1 == bt1 * D)) { /* single bin */
    acc_add(A, bt0, k * (double)(t1 - t0));
    return;
  }
  int64_t bf = bt0, bl = bt1;
  if (t0 != bt0 * D) { acc_add(A, bt0, k * (double)((bt0 + 1) * D - t0)); bf = bt0 + 1; }
  if (t1 != bt1 * D) acc_add(A, bt1, k * (double)(t1 - bt1 * D));
  /* whole bins [bf, bl) */
  if (bf < A->b0) bf = A->b0;
  if (bl > A->b1) bl = A->b1;
  if (bf < bl) {
    A->diff[bf - A->b0] += k * (double)D;
    A->diff[bl - A->b0] -= k * (double)D;
  }
}

/* Per-pin state of the clock-cycle glitch detection. */
typedef struct {
  int64_t cyc;      /* clock cycle of the pin's last event (-1: none yet) */
  int64_t last_t;   /* time of the pin's last event */
  float last_slew;  /* slew of the pin's last event */
  int cnt;          /* events of the pin in cycle cyc */
} pin_glitch;

/* GlitchDetectUpdate for one event of a pin at time t with slew `slew`:
 * returns the glitch scaling ratio r > 0 when the event is not the pin's
 * first in its clock cycle, else -1 (a regular event). */
static double glitch_update(const orc_problem* P, pin_glitch* s, int64_t t, float slew) {
  const int64_t cyc = t / P->glitch_clk;
  if (s->cyc != cyc) {
    s->cyc = cyc;
    s->cnt = 0;
  }
  s->cnt += 1;
  double r = -1.0;
  if (s->cnt > 1) {
    const double pw = (double)(t - s->last_t);
#if ORC_PLANT == 11
    const double q = pw / ((double)slew + (double)s->last_slew); /* planted: dropped factor 2 */
#else
    const double q = 2.0 * pw / ((double)slew + (double)s->last_slew);
#endif
    r = q * q < 1.0 ? q * q : 1.0;
  }
  s->last_t = t;
  s->last_slew = slew;
  return r;
}

/* Evaluate one gate (Algorithm 1 order). trace arrays may be NULL.
 * tot: [E_int, E_sw, E_leak, E_gl] of the gate are added to it. */
static int eval_gate(const orc_problem* P, int64_t g, acc_t* A, double* tot, int32_t* st_before,
                     int64_t* bin_out, int64_t* bad) {
  const int32_t c = P->gate_cell[g];
  const int32_t I = P->n_inputs[c];
  /* the state index: input pins, or all pins (bit I = output) */
#if ORC_PLANT == 13
  const uint32_t smask = low_bits(I); /* planted: the output pin left out of an all-pin state */
#else
  const uint32_t smask = low_bits(P->state_all_pins ? I + 1 : I);
#endif
  pin_glitch pg[32];
  for (int p = 0; p < 32; ++p) {
    pg[p].cyc = -1;
    pg[p].last_t = 0;
    pg[p].last_slew = 0.f;
    pg[p].cnt = 0;
  }
  const double C = P->net_load[P->gate_out_net[g]];
  const double lam = P->leak_scale ? P->leak_scale[g] : 1.0;
  uint32_t vals = P->gate_init[g] & low_bits(I + 1);
  int64_t t_prev = 0;
  const int64_t e_end = P->gate_off[g + 1];
  int64_t e = P->gate_off[g];
  while (e < e_end) {
    const int64_t t = P->t[e];
    if (t < 0 || t >= P->t_end) { *bad = e; return ORC_ERR_EVENT_RANGE; }
    if (t < t_prev) { *bad = e; return ORC_ERR_EVENT_ORDER; }
    int64_t e2 = e + 1;
    while (e2 < e_end && P->t[e2] == t) ++e2;
    const uint32_t s = vals & smask; /* input state before the group */
    /* 1. leakage of [t_prev, t) at the state held over it */
#if ORC_PLANT == 4
    {
      /* planted: interval charged at the state after the group */
      uint32_t v2 = vals;
      for (int64_t q = e; q < e2; ++q) {
        int p = P->pin_bit[q] >> 1, v = P->pin_bit[q] & 1;
        v2 = (v2 & ~(1u << p)) | ((uint32_t)v << p);
      }
      double r = lam * leak_value(P, c, v2 & smask);
      add_leak(P, A, t_prev, t, r);
      tot[2] += r * 1e-6 * (double)(t - t_prev);
    }
#else
    {
      double r = lam * leak_value(P, c, s);
      add_leak(P, A, t_prev, t, r);
      tot[2] += r * 1e-6 * (double)(t - t_prev);
    }
#endif
    /* 2. dynamic energy of each event of the group, all at the group-start state */
    uint32_t seen = 0;
#if ORC_PLANT == 1
    uint32_t cur = vals; /* planted: intermediate state inside a group */
#endif
    for (int64_t q = e; q < e2; ++q) {
      const int p = P->pin_bit[q] >> 1, v = P->pin_bit[q] & 1;
      if (p > I) { *bad = q; return ORC_ERR_EVENT_RANGE; }
      if ((seen >> p) & 1u) { *bad = q; return ORC_ERR_EVENT_ORDER; }
      if ((int)((vals >> p) & 1u) == v) { *bad = q; return ORC_ERR_NOT_TOGGLE; }
      seen |= 1u << p;
#if ORC_PLANT == 1
      const uint32_t sl = cur & smask;
      cur = (cur & ~(1u << p)) | ((uint32_t)v << p);
#else
      const uint32_t sl = s;
#endif
#if ORC_PLANT == 7
      const int dir = !v; /* planted: wrong direction table */
#else
      const int dir = v;
#endif
      const int32_t k = table_id(P, c, sl, dir);
      const double ei = orc_bilerp(P, c, k, (double)P->slew[q], C);
      const double es = (p == I) ? sw_energy(P, C, v) : 0.0;
      const int64_t b = bin_of(P, t);
      const double r = P->glitch_clk > 0 ? glitch_update(P, &pg[p], t, P->slew[q]) : -1.0;
      if (r > 0.0) {
#if ORC_PLANT == 12
        acc_add(A, b, ei + es); /* planted: glitch energy not scaled in the waveform */
#else
        acc_add(A, b, r * (ei + es));
#endif
        tot[3] += r * (ei + es);
      } else {
        acc_add(A, b, ei + es);
        tot[0] += ei;
        tot[1] += es;
      }
      if (st_before) st_before[q] = (int32_t)sl;
      if (bin_out) bin_out[q] = b;
    }
    /* 3. apply the group */
    for (int64_t q = e; q < e2; ++q) {
      const int p = P->pin_bit[q] >> 1, v = P->pin_bit[q] & 1;
      vals = (vals & ~(1u << p)) | ((uint32_t)v << p);
    }
    t_prev = t;
    e = e2;
  }
#if ORC_PLANT != 6
  {
    double r = lam * leak_value(P, c, vals & smask);
    add_leak(P, A, t_prev, P->t_end, r);
    tot[2] += r * 1e-6 * (double)(P->t_end - t_prev);
  }
#endif
  return ORC_OK;
}

int orc_forward(const orc_problem* P, int64_t b0, int64_t b1, int leak_mode, const int64_t* gates,
                int64_t n_gate_list, double* E, double* totals, int nthreads, int64_t* bad_event) {
  if (!P || !E || b0 < 0 || b1 < b0 || b1 > orc_num_bins(P) || P->bin_ps <= 0) return ORC_ERR_INVALID_ARG;
  if (check_patterns(P) != ORC_OK) return ORC_ERR_INVALID_ARG;
  const int64_t nb = b1 - b0;
  const int64_t ng = gates ? n_gate_list : P->n_gates;
  int nt = nthreads > 0 ? nthreads : orc_max_threads();
  if (nt < 1) nt = 1;
  memset(E, 0, sizeof(double) * (size_t)nb);
  double tot_all[4] = {0, 0, 0, 0};
  int status = ORC_OK;
  int64_t bad = -1;
#pragma omp parallel num_threads(nt)
  {
    acc_t A;
    A.b0 = b0; A.b1 = b1; A.mode = leak_mode;
    A.E = (double*)calloc((size_t)(nb > 0 ? nb : 1), sizeof(double));
    A.diff = (double*)calloc((size_t)nb + 1, sizeof(double));
    double tot[4] = {0, 0, 0, 0};
    int st = (A.E && A.diff) ? ORC_OK : ORC_ERR_INVALID_ARG;
    int64_t mybad = -1;
#pragma omp for schedule(dynamic, 64)
    for (int64_t q = 0; q < ng; ++q) {
      if (st != ORC_OK) continue;
      int64_t g = gates ? gates[q] : q;
      if (g < 0 || g >= P->n_gates) { st = ORC_ERR_INVALID_ARG; continue; }
      st = eval_gate(P, g, &A, tot, NULL, NULL, &mybad);
    }
    if (A.mode == 1 && A.E && A.diff) {
      double run = 0;
      for (int64_t b = 0; b < nb; ++b) { run += A.diff[b]; A.E[b] += run; }
    }
#pragma omp critical
    {
      if (st != ORC_OK && status == ORC_OK) { status = st; bad = mybad; }
      if (A.E)
        for (int64_t b = 0; b < nb; ++b) E[b] += A.E[b];
      for (int q = 0; q < 4; ++q) tot_all[q] += tot[q];
    }
    free(A.E);
    free(A.diff);
  }
  if (totals) { totals[0] = tot_all[0]; totals[1] = tot_all[1]; totals[2] = tot_all[2]; totals[3] = tot_all[3]; }
  if (bad_event) *bad_event = bad;
  return status;
}

int orc_event_trace(const orc_problem* P, int32_t* state_before, int64_t* bin, int64_t* bad_event) {
  if (!P || !state_before || !bin || check_patterns(P) != ORC_OK) return ORC_ERR_INVALID_ARG;
  acc_t A;
  double dummy = 0;
  A.b0 = 0; A.b1 = 0; A.mode = 0; A.E = &dummy; A.diff = NULL;
  double tot[4] = {0, 0, 0, 0};
  for (int64_t g = 0; g < P->n_gates; ++g) {
    int64_t bad = -1;
    int st = eval_gate(P, g, &A, tot, state_before, bin, &bad);
    if (st != ORC_OK) { if (bad_event) *bad_event = bad; return st; }
  }
  return ORC_OK;
}

int orc_gate_report(const orc_problem* P, double* gate_e, int64_t* t_max, int nthreads) {
  if (!P || !gate_e || !t_max || check_patterns(P) != ORC_OK) return ORC_ERR_INVALID_ARG;
  int nt = nthreads > 0 ? nthreads : orc_max_threads();
  int status = ORC_OK;
  int64_t tm = -1;
#pragma omp parallel for schedule(dynamic, 64) num_threads(nt) reduction(max : tm)
  for (int64_t g = 0; g < P->n_gates; ++g) {
    acc_t A;
    double dummy = 0;
    A.b0 = 0; A.b1 = 0; A.mode = 0; A.E = &dummy; A.diff = NULL;
    double tot[4] = {0, 0, 0, 0};
    int64_t bad = -1;
    if (eval_gate(P, g, &A, tot, NULL, NULL, &bad) != ORC_OK) {
#pragma omp critical
      status = ORC_ERR_INVALID_ARG;
    }
    gate_e[4 * g + 0] = tot[2];
    gate_e[4 * g + 1] = tot[0];
    gate_e[4 * g + 2] = tot[1];
    gate_e[4 * g + 3] = tot[3];
    if (P->gate_off[g + 1] > P->gate_off[g] && P->t[P->gate_off[g + 1] - 1] > tm) tm = P->t[P->gate_off[g + 1] - 1];
  }
  *t_max = tm;
  return status;
}

int orc_validate(const orc_problem* P, int64_t* bad_event) {
  if (!P || check_patterns(P) != ORC_OK) return ORC_ERR_INVALID_ARG;
  acc_t A;
  double dummy = 0;
  A.b0 = 0; A.b1 = 0; A.mode = 0; A.E = &dummy; A.diff = NULL;
  double tot[4] = {0, 0, 0, 0};
  for (int64_t g = 0; g < P->n_gates; ++g) {
    int64_t bad = -1;
    int st = eval_gate(P, g, &A, tot, NULL, NULL, &bad);
    if (st != ORC_OK) { if (bad_event) *bad_event = bad; return st; }
  }
  if (bad_event) *bad_event = -1;
  return ORC_OK;
}

/*
 * Adjoint. With P_b = E_b / D and gP[b] = dL/dP_b:
 *   dL/dC_g  = sum over g's events e of gP[bin(e)]/D * (dE_int/dC + dE_sw/dC)
 *   dL/dlam_g = sum over g's intervals [t0,t1) at state s of
 *               leak[s] * 1e-6 * sum_b gP[b]/D * |[t0,t1) ∩ bin b|
 * The inner bin sum is evaluated bin by bin (leak_mode 0) or as the
 * difference of the cumulative integral of the piecewise-constant function
 * gP[floor(t/D)]/D (leak_mode 1); both are the same quantity.
 */
static double cum_g(const orc_problem* P, const double* PG, const double* gP, int64_t nb, int64_t t) {
  const int64_t D = P->bin_ps;
  int64_t b = t / D;
  if (b >= nb) return PG[nb];
  return PG[b] + gP[b] * (double)(t - b * D) / (double)D;
}

static double interval_gsum(const orc_problem* P, const double* PG, const double* gP, int64_t nb, int mode,
                            int64_t t0, int64_t t1) {
  if (t1 <= t0) return 0.0;
  const int64_t D = P->bin_ps;
  if (mode == 1) return cum_g(P, PG, gP, nb, t1) - cum_g(P, PG, gP, nb, t0);
  double s = 0;
  for (int64_t b = t0 / D; b <= (t1 - 1) / D; ++b) {
    int64_t lo = b * D > t0 ? b * D : t0;
    int64_t hi = (b + 1) * D < t1 ? (b + 1) * D : t1;
#if ORC_PLANT == 10
    if (hi - lo < D) continue; /* planted: partial bins dropped */
#endif
    s += gP[b] * (double)(hi - lo) / (double)D;
  }
  return s;
}

int orc_adjoint(const orc_problem* P, const double* gP, int leak_mode, double* grad_load, double* grad_scale,
                int nthreads) {
  if (!P || !gP || !grad_load || !grad_scale || check_patterns(P) != ORC_OK) return ORC_ERR_INVALID_ARG;
  const int64_t nb = orc_num_bins(P);
  const double D = (double)P->bin_ps;
  double* PG = (double*)malloc(sizeof(double) * (size_t)(nb + 1));
  if (!PG) return ORC_ERR_INVALID_ARG;
  PG[0] = 0;
  for (int64_t b = 0; b < nb; ++b) PG[b + 1] = PG[b] + gP[b];
  memset(grad_load, 0, sizeof(double) * (size_t)P->n_nets);
  memset(grad_scale, 0, sizeof(double) * (size_t)P->n_gates);
  double* gC = (double*)calloc((size_t)(P->n_gates > 0 ? P->n_gates : 1), sizeof(double));
  if (!gC) { free(PG); return ORC_ERR_INVALID_ARG; }
  int nt = nthreads > 0 ? nthreads : orc_max_threads();
  int status = ORC_OK;
#pragma omp parallel for schedule(dynamic, 64) num_threads(nt)
  for (int64_t g = 0; g < P->n_gates; ++g) {
    const int32_t c = P->gate_cell[g];
    const int32_t I = P->n_inputs[c];
    const uint32_t smask = low_bits(P->state_all_pins ? I + 1 : I);
    const double C = P->net_load[P->gate_out_net[g]];
    uint32_t vals = P->gate_init[g] & low_bits(I + 1);
    int64_t t_prev = 0;
    double dC = 0, dl = 0;
    pin_glitch pg[32];
    for (int p = 0; p < 32; ++p) {
      pg[p].cyc = -1;
      pg[p].last_t = 0;
      pg[p].last_slew = 0.f;
      pg[p].cnt = 0;
    }
    int64_t e = P->gate_off[g];
    const int64_t e_end = P->gate_off[g + 1];
    while (e < e_end) {
      const int64_t t = P->t[e];
      int64_t e2 = e + 1;
      while (e2 < e_end && P->t[e2] == t) ++e2;
      const uint32_t s = vals & smask;
      dl += leak_value(P, c, s) * 1e-6 * interval_gsum(P, PG, gP, nb, leak_mode, t_prev, t);
      const int64_t b = t / P->bin_ps;
      for (int64_t q = e; q < e2; ++q) {
        const int p = P->pin_bit[q] >> 1, v = P->pin_bit[q] & 1;
        const int32_t k = table_id(P, c, s, v);
        double d = bilerp_dload(P, c, k, (double)P->slew[q], C);
        if (p == I) d += sw_energy_dC(P, v);
        if (P->glitch_clk > 0) {
          const double r = glitch_update(P, &pg[p], t, P->slew[q]);
          if (r > 0.0) d *= r;
        }
        dC += gP[b] / D * d;
      }
      for (int64_t q = e; q < e2; ++q) {
        const int p = P->pin_bit[q] >> 1, v = P->pin_bit[q] & 1;
        vals = (vals & ~(1u << p)) | ((uint32_t)v << p);
      }
      t_prev = t;
      e = e2;
    }
    dl += leak_value(P, c, vals & smask) * 1e-6 * interval_gsum(P, PG, gP, nb, leak_mode, t_prev, P->t_end);
    gC[g] = dC;
    grad_scale[g] = dl;
  }
  for (int64_t g = 0; g < P->n_gates; ++g) grad_load[P->gate_out_net[g]] += gC[g];
  free(gC);
  free(PG);
  return status;
}
