/*
 * Seeded synthetic workload generator for gate-level toggle-event traces.
 *
 * This module produces INPUTS only: a standard-cell power library, a netlist
 * and per-gate toggle-event streams. It contains none of the power method's
 * arithmetic (no state lookup, interpolation, energy, leakage or binning);
 * both the FP64 reference evaluator and the GPU library consume its output.
 *
 * Workload shapes follow the paper's setting (Sec. 6.1 designs; Sec. 3.2:
 * heavy-tailed per-gate event counts, p90/p99 orders of magnitude above p50)
 * with the sizes of the synthetic configurations stated in the design doc.
 *
 * Random numbers: a counter-based generator. Each draw is a pure function of
 * (seed, stream, index) built from the SplitMix64 output finaliser (Steele,
 * Lea & Flood, "Fast splittable pseudorandom number generators", OOPSLA
 * 2014), so results are independent of thread count and order.
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC synth.c -o libsynth.so -lm
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define SYN_OK 0
#define SYN_ERR_ARG 1
#define SYN_ERR_RANGE 2

/* streams */
enum { ST_LIB = 1, ST_NET = 2, ST_CNT = 3, ST_TIME = 4, ST_PIN = 5, ST_SLEW = 6, ST_INIT = 7, ST_TIE = 8, ST_LOAD = 9 };

static inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

/* draw number `idx` of stream `stream` under `seed` */
static inline uint64_t draw(uint64_t seed, uint64_t stream, uint64_t idx) {
  uint64_t k = mix64(seed * 0x9E3779B97F4A7C15ULL + stream * 0xD1B54A32D192ED03ULL + 0x632BE59BD9B4E019ULL);
  return mix64(k ^ (idx * 0x9E3779B97F4A7C15ULL + 0x8CB92BA72F3D8DD7ULL));
}

/* uniform in [0,1) from the top 53 bits */
static inline double unif(uint64_t seed, uint64_t stream, uint64_t idx) {
  return (double)(draw(seed, stream, idx) >> 11) * (1.0 / 9007199254740992.0);
}

/* uniform integer in [0, n) */
static inline uint64_t unif_int(uint64_t seed, uint64_t stream, uint64_t idx, uint64_t n) {
  return (uint64_t)(unif(seed, stream, idx) * (double)n);
}

/* standard normal by Box-Muller from two uniforms of the stream */
static inline double normal(uint64_t seed, uint64_t stream, uint64_t idx) {
  double u1 = unif(seed, stream, 2 * idx);
  double u2 = unif(seed, stream, 2 * idx + 1);
  if (u1 < 1e-300) u1 = 1e-300;
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586476925 * u2);
}

/* Number of inputs per cell: U{1..i_max}. */
int synth_cell_inputs(uint64_t seed, int32_t n_cells, int32_t i_max, int32_t* n_inputs) {
  if (n_cells <= 0 || i_max < 1 || i_max > 16 || !n_inputs) return SYN_ERR_ARG;
  for (int32_t c = 0; c < n_cells; ++c)
    n_inputs[c] = 1 + (int32_t)unif_int(seed, ST_LIB, (uint64_t)c, (uint64_t)i_max);
  return SYN_OK;
}

/*
 * Library tables. Axes are shared by every cell and geometric:
 *   slew_i = slew_lo * (slew_hi/slew_lo)^(i/(n_slew-1)),   load likewise.
 * Every (state, direction) pair gets its own table (identity state map):
 *   local table id = 2*state + dir, dir 0 = falling, 1 = rising.
 * Table entries: e0 + e1*(s/100) + e2*(C/10) + e3*sqrt((s/100)*(C/10)),
 * e* ~ U(0.05, 2) fJ per table (positive, monotone, not bilinear).
 * Leakage per (cell, state) ~ U(leak_lo, leak_hi) nW.
 * Output arrays are sized by the caller from n_inputs:
 *   map entries   = sum_c 2 * 2^I_c   (int16)
 *   tables        = sum_c 2 * 2^I_c   (each n_slew*n_load floats)
 *   leak entries  = sum_c 2^I_c
 */
int synth_library(uint64_t seed, int32_t n_cells, int32_t n_slew, int32_t n_load, const int32_t* n_inputs,
                  double slew_lo, double slew_hi, double load_lo, double load_hi, double leak_lo, double leak_hi,
                  float* slew_axis, float* load_axis, int64_t* map_base, int16_t* state_to_table,
                  int64_t* table_base, float* tables, int64_t* leak_base, float* leak) {
  if (n_cells <= 0 || n_slew < 2 || n_load < 2 || !n_inputs) return SYN_ERR_ARG;
  int64_t mb = 0, tb = 0, lb = 0;
  uint64_t rix = 1000000;  /* draw index space for table coefficients */
  for (int32_t c = 0; c < n_cells; ++c) {
    int32_t I = n_inputs[c];
    int64_t ns = (int64_t)1 << I;
    for (int32_t i = 0; i < n_slew; ++i)
      slew_axis[(int64_t)c * n_slew + i] = (float)(slew_lo * pow(slew_hi / slew_lo, (double)i / (n_slew - 1)));
    for (int32_t j = 0; j < n_load; ++j)
      load_axis[(int64_t)c * n_load + j] = (float)(load_lo * pow(load_hi / load_lo, (double)j / (n_load - 1)));
    map_base[c] = mb;
    table_base[c] = tb;
    leak_base[c] = lb;
    for (int64_t s = 0; s < ns; ++s) {
      for (int d = 0; d < 2; ++d) {
        state_to_table[mb + 2 * s + d] = (int16_t)(2 * s + d);
        double e[4];
        for (int q = 0; q < 4; ++q) e[q] = 0.05 + 1.95 * unif(seed, ST_LIB, rix++);
        float* T = tables + (tb + 2 * s + d) * (int64_t)n_slew * n_load;
        for (int32_t i = 0; i < n_slew; ++i) {
          double sv = slew_axis[(int64_t)c * n_slew + i] / 100.0;
          for (int32_t j = 0; j < n_load; ++j) {
            double cv = load_axis[(int64_t)c * n_load + j] / 10.0;
            T[i * n_load + j] = (float)(e[0] + e[1] * sv + e[2] * cv + e[3] * sqrt(sv * cv));
          }
        }
      }
      leak[lb + s] = (float)(leak_lo + (leak_hi - leak_lo) * unif(seed, ST_LIB, rix++));
    }
    mb += 2 * ns;
    tb += 2 * ns;
    lb += ns;
  }
  return SYN_OK;
}

/*
 * Netlist: gate g takes cell U{0..n_cells-1}; n_pi primary-input nets come
 * first and gate g drives net n_pi + g. Net loads ~ U(load_lo, load_hi) fF
 * (primary inputs included, unused by any gate as an output). Initial pin
 * values: bit p of gate_init = value of pin p (inputs 0..I-1, output I).
 */
int synth_netlist(uint64_t seed, int64_t n_gates, int32_t n_cells, const int32_t* n_inputs, int64_t n_pi,
                  double load_lo, double load_hi, int32_t* gate_cell, int32_t* gate_out_net, uint32_t* gate_init,
                  float* net_load) {
  if (n_gates < 0 || n_cells <= 0 || n_pi < 0) return SYN_ERR_ARG;
#pragma omp parallel for schedule(static)
  for (int64_t g = 0; g < n_gates; ++g) {
    int32_t c = (int32_t)unif_int(seed, ST_NET, (uint64_t)g, (uint64_t)n_cells);
    gate_cell[g] = c;
    gate_out_net[g] = (int32_t)(n_pi + g);
    uint32_t npins = (uint32_t)n_inputs[c] + 1;
    gate_init[g] = (uint32_t)(draw(seed, ST_INIT, (uint64_t)g) & ((1ULL << npins) - 1));
  }
  int64_t n_nets = n_pi + n_gates;
#pragma omp parallel for schedule(static)
  for (int64_t n = 0; n < n_nets; ++n)
    net_load[n] = (float)(load_lo + (load_hi - load_lo) * unif(seed, ST_LOAD, (uint64_t)n));
  return SYN_OK;
}

/* clock gates: evenly spread indices floor(k*G/n_clock) */
int synth_is_clock(int64_t n_gates, int64_t n_clock, uint8_t* is_clock) {
  if (n_clock < 0 || n_clock > n_gates) return SYN_ERR_ARG;
  memset(is_clock, 0, (size_t)n_gates);
  for (int64_t k = 0; k < n_clock; ++k) is_clock[(k * n_gates) / n_clock] = 1;
  return SYN_OK;
}

typedef struct { double frac; int64_t g; } rem_t;
static int cmp_rem(const void* a, const void* b) {
  const rem_t* x = (const rem_t*)a; const rem_t* y = (const rem_t*)b;
  if (x->frac > y->frac) return -1;
  if (x->frac < y->frac) return 1;
  return (x->g < y->g) ? -1 : (x->g > y->g);
}

/*
 * Per-gate event counts. Clock gates get clock_events each. The other gates
 * draw weights from the distribution (dist 0: lognormal(p1, p2); dist 1:
 * rank-Zipf with exponent p1 over a seeded random rank permutation;
 * dist 2: all weights equal) and `total_other` events are apportioned by the
 * largest-remainder method, so the grand total is exact. Fails with
 * SYN_ERR_RANGE if any count exceeds max_per_gate.
 */
int synth_counts(uint64_t seed, int64_t n_gates, const uint8_t* is_clock, int64_t clock_events, int32_t dist,
                 double p1, double p2, int64_t total_other, int64_t max_per_gate, int64_t* counts) {
  if (n_gates < 0 || total_other < 0) return SYN_ERR_ARG;
  int64_t n_other = 0;
  for (int64_t g = 0; g < n_gates; ++g) n_other += !is_clock[g];
  if (n_other == 0 && total_other > 0) return SYN_ERR_ARG;
  double* w = (double*)malloc(sizeof(double) * (size_t)(n_gates > 0 ? n_gates : 1));
  if (!w) return SYN_ERR_ARG;
  if (dist == 1) {
    /* rank permutation: sort gates by a hash key; rank r gets weight (r+1)^-s */
    rem_t* key = (rem_t*)malloc(sizeof(rem_t) * (size_t)(n_gates > 0 ? n_gates : 1));
    if (!key) { free(w); return SYN_ERR_ARG; }
    for (int64_t g = 0; g < n_gates; ++g) { key[g].frac = unif(seed, ST_CNT, (uint64_t)g); key[g].g = g; }
    qsort(key, (size_t)n_gates, sizeof(rem_t), cmp_rem);
    int64_t r = 0;
    for (int64_t q = 0; q < n_gates; ++q) {
      int64_t g = key[q].g;
      if (is_clock[g]) { w[g] = 0; continue; }
      w[g] = pow((double)(r + 1), -p1);
      ++r;
    }
    free(key);
  } else {
#pragma omp parallel for schedule(static)
    for (int64_t g = 0; g < n_gates; ++g) {
      if (is_clock[g]) { w[g] = 0; continue; }
      w[g] = (dist == 0) ? exp(p1 + p2 * normal(seed, ST_CNT, (uint64_t)g)) : 1.0;
    }
  }
  double wsum = 0;
  for (int64_t g = 0; g < n_gates; ++g) wsum += w[g];
  rem_t* rem = (rem_t*)malloc(sizeof(rem_t) * (size_t)(n_other > 0 ? n_other : 1));
  if (!rem) { free(w); return SYN_ERR_ARG; }
  int64_t assigned = 0, q = 0;
  for (int64_t g = 0; g < n_gates; ++g) {
    if (is_clock[g]) { counts[g] = clock_events; continue; }
    double raw = (wsum > 0) ? (double)total_other * w[g] / wsum : 0.0;
    double fl = floor(raw);
    counts[g] = (int64_t)fl;
    assigned += counts[g];
    rem[q].frac = raw - fl; rem[q].g = g; ++q;
  }
  int64_t left = total_other - assigned;
  if (left > 0) qsort(rem, (size_t)n_other, sizeof(rem_t), cmp_rem);
  for (int64_t k = 0; k < left; ++k) counts[rem[k % n_other].g] += 1;
  free(rem);
  free(w);
  for (int64_t g = 0; g < n_gates; ++g)
    if (counts[g] > max_per_gate) return SYN_ERR_RANGE;
  return SYN_OK;
}

/*
 * Event streams, gate-major CSR (gate_off = exclusive prefix of counts), each
 * gate's events sorted by time and merged across its pins.
 *   Clock gates toggle input pin 0 at t = k*t_clk/2, k = 1..count.
 *   Other gates: integer stratified jitter over [0, t_end):
 *     a_k = floor(k*t_end/N), t_k = a_k + floor(u_k*(a_{k+1}-a_k)),
 *   strictly increasing when N <= t_end. Pin ~ U{0..I} (I = output pin);
 *   the new value alternates per pin starting from the gate's initial value.
 *   With probability p_tie an event instead takes the previous event's time
 *   (a simultaneous event) when its pin is not already used at that time.
 *   Slews ~ U(slew_lo, slew_hi) ps.
 * pin_bit = (pin << 1) | new_value.
 */
int synth_events(uint64_t seed, int64_t n_gates, const int32_t* gate_cell, const int32_t* n_inputs,
                 const uint32_t* gate_init, const uint8_t* is_clock, const int64_t* gate_off, int64_t t_end,
                 int64_t t_clk, double p_tie, double slew_lo, double slew_hi, int64_t* t, uint8_t* pin_bit,
                 float* slew) {
  if (n_gates < 0 || t_end <= 0) return SYN_ERR_ARG;
  int err = 0;
#pragma omp parallel for schedule(dynamic, 256) reduction(| : err)
  for (int64_t g = 0; g < n_gates; ++g) {
    int64_t o = gate_off[g], n = gate_off[g + 1] - o;
    if (n == 0) continue;
    int32_t I = n_inputs[gate_cell[g]];
    uint32_t val = gate_init[g];
    if (is_clock && is_clock[g]) {
      for (int64_t k = 0; k < n; ++k) {
        int64_t tk = (k + 1) * t_clk / 2;
        if (tk >= t_end) err |= 1;
        t[o + k] = tk;
        uint32_t nv = ((val >> 0) & 1u) ^ 1u;
        val = (val & ~1u) | nv;
        pin_bit[o + k] = (uint8_t)((0 << 1) | nv);
        slew[o + k] = (float)(slew_lo + (slew_hi - slew_lo) * unif(seed, ST_SLEW, (uint64_t)(o + k)));
      }
      continue;
    }
    if (n > t_end) { err |= 1; continue; }
    uint32_t group_pins = 0;
    int64_t prev_t = -1;
    for (int64_t k = 0; k < n; ++k) {
      uint64_t e = (uint64_t)(o + k);
      int64_t a0 = (int64_t)(((__int128)k * t_end) / n);
      int64_t a1 = (int64_t)(((__int128)(k + 1) * t_end) / n);
      int64_t tk = a0 + (int64_t)(unif(seed, ST_TIME, e) * (double)(a1 - a0));
      int32_t pin = (int32_t)unif_int(seed, ST_PIN, e, (uint64_t)(I + 1));
      if (k > 0 && p_tie > 0 && unif(seed, ST_TIE, e) < p_tie && !((group_pins >> pin) & 1u)) tk = prev_t;
      if (tk != prev_t) group_pins = 0;
      group_pins |= 1u << pin;
      uint32_t nv = ((val >> pin) & 1u) ^ 1u;
      val = (val & ~(1u << pin)) | (nv << pin);
      t[e] = tk;
      pin_bit[e] = (uint8_t)((pin << 1) | (int32_t)nv);
      slew[e] = (float)(slew_lo + (slew_hi - slew_lo) * unif(seed, ST_SLEW, e));
      prev_t = tk;
    }
  }
  return err ? SYN_ERR_RANGE : SYN_OK;
}

/* utility for tests: raw 64-bit draws */
int synth_draws(uint64_t seed, uint64_t stream, uint64_t start, int64_t n, uint64_t* out) {
  for (int64_t i = 0; i < n; ++i) out[i] = draw(seed, stream, start + (uint64_t)i);
  return SYN_OK;
}

/*
 * Time window [t0, t1) of a gate-major CSR trace (times sorted within each
 * gate): out_off[G+1] and the window's events (absolute times), in gate
 * order. Pass out arrays NULL to get only out_off (the count); *n_out = the
 * window's events.
 */
static int64_t lower_bound_t(const int64_t* t, int64_t lo, int64_t hi, int64_t x) {
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (t[mid] < x) lo = mid + 1; else hi = mid;
  }
  return lo;
}

int synth_window(int64_t n_gates, const int64_t* gate_off, const int64_t* t, const uint8_t* pin_bit,
                 const float* slew, int64_t t0, int64_t t1, int64_t* out_off, int64_t* out_t, uint8_t* out_pb,
                 float* out_slew, int64_t* n_out) {
  if (n_gates < 0 || t1 < t0 || !gate_off || !out_off) return SYN_ERR_ARG;
  out_off[0] = 0;
#pragma omp parallel for schedule(static)
  for (int64_t g = 0; g < n_gates; ++g) {
    int64_t a = lower_bound_t(t, gate_off[g], gate_off[g + 1], t0);
    int64_t b = lower_bound_t(t, a, gate_off[g + 1], t1);
    out_off[g + 1] = b - a;
  }
  for (int64_t g = 0; g < n_gates; ++g) out_off[g + 1] += out_off[g];
  if (n_out) *n_out = out_off[n_gates];
  if (!out_t) return SYN_OK;
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t g = 0; g < n_gates; ++g) {
    int64_t a = lower_bound_t(t, gate_off[g], gate_off[g + 1], t0);
    int64_t n = out_off[g + 1] - out_off[g];
    memcpy(out_t + out_off[g], t + a, (size_t)n * 8);
    memcpy(out_pb + out_off[g], pin_bit + a, (size_t)n);
    memcpy(out_slew + out_off[g], slew + a, (size_t)n * 4);
  }
  return SYN_OK;
}
