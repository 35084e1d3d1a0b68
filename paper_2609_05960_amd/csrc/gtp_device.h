// Device side of the binned power-waveform library (gfx950, wave64).
//
// Data layout in HBM (all struct-of-arrays):
//   events   the caller's gate-major CSR arrays: t int64, pin_bit uint8
//            ((pin << 1) | new value), slew float, gate_off int64[G+1]
//            (borrowed), and the library's packed copy of them (built once
//            per event set and bin width; see gtp_pack.h): per time tile,
//            "units" of at most 16 consecutive events of one gate, 64 units
//            per wavefront group, events stored unit-interleaved so that the
//            k-th events of a group's units are adjacent;
//   library  per cell a meta record, the (state, dir) -> table map stored as
//            the table's first quad index, leakage values, slew axis and
//            reciprocal segment widths (staged in LDS by every kernel), and
//            the tables as "quads": for table T and axis cell (i, j) the four
//            corners (T[i][j], T[i][j+1], T[i+1][j], T[i+1][j+1]) as one
//            16-byte vector, so an interpolation is one 16-byte gather;
//   gates    per call, a 16-byte parameter record per gate (load-axis
//            segment and weight, switching energy, leakage scale);
//   bins     int64 fixed-point accumulators X (energy) and S (leakage steps).
//
// Fixed point. With E = 2^-m fJ the energy unit and R = 1e6 * 2^-m nW the
// leakage-rate unit (so that R * 1 ps = E), every contribution is an integer
// and sums are exact and independent of the order of accumulation. An event
// energy e (FP32, fJ) becomes e * 2^m exactly (split into two 32-bit halves,
// see energy_fixed). The leakage rate of a gate in input state s is quantised
// once, q = rint(lambda * leak[s] * 2^m * 1e-6) (FP32), and every input event
// adds the step q(after) - q(before): per gate the steps telescope exactly, so
// the rate at any time is exactly the quantised rate of the state held.
//
// Leakage in step form (an exact rewrite of the interval rule of Sec. 2.4,
// Eq. leakage energy): with R(t) = sum_g q_g(s_g(t)) the total rate, the
// leakage energy of bin b is  D * R(b*D) + sum over steps d at time t in bin b
// of d * ((b+1)*D - t).  So each input event contributes its step d to S[b]
// and d * ((b+1)*D - t) to X[b]; a prefix sum of S gives R at bin starts.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gtp {

constexpr int kLaneEvents = 16;       // events per lane block / per unit (max)
constexpr int kFwdThreads = 256;      // threads of the gate-major walking kernels
constexpr int kTileThreads = 1024;    // threads of the packed forward kernel (default)
constexpr int kGroupUnits = 64;       // units per wavefront group (one per lane)
constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

// Packed event record (three 32-bit words, built once per event set, bin
// width and library; everything in it is independent of the per-call loads
// and leakage scales):
//   word  bits [0, 23) in-tile time (bin_in_tile << r_bits | r), [23, 31)
//         the leakage entry of the gate's state after the event, relative to
//         the cell's first (the state itself for a kCellDirect cell, its
//         leakage item for a wider one): the leakage held from the event on;
//   row   bits [0, 30) the quad index of the event's table row at its slew
//         segment, i.e. map(state before the timestamp group, new value) +
//         segment * (n_load - 1), to which the gate's load segment is added;
//         bit 30 set for an output event, bit 31 the new value;
//   alpha the slew weight (slew - S[i]) / (S[i+1] - S[i]) in FP32, rounded
//         as the gate-major kernels round it.
// With glitch detection on, a fourth word per event holds its energy factor
// (the glitch scaling ratio of a glitch event, 1 otherwise).
constexpr int kTimeBits = 23;
constexpr uint32_t kTimeMask = (1u << kTimeBits) - 1u;
constexpr int kStateShift = 23;
constexpr uint32_t kRowMask = (1u << 30) - 1u;
constexpr int kOutBit = 30;

// Per-cell record staged in LDS. How a state selects the cell's table and
// leakage value (Sec. 4.1):
//   kCellDirect  a per-state array in the LDS image (at most 8 state pins):
//                entry (s, dir) at map_off + 2*s + dir, leakage at leak_off + s;
//   kCellSipl    per-state item arrays in device memory (9..16 state pins):
//                item k = sipl[t_sipl + s] (tables), sipl[l_sipl + s]
//                (leakage), entry (k, dir) at map_off + 2*k + dir, leakage
//                at leak_off + k;
//   kCellScan    the state patterns themselves (more than 16 state pins): k
//                = the first pattern whose care pins agree with s, scanned
//                in device memory, then as kCellSipl.
constexpr int kCellDirect = 0, kCellSipl = 1, kCellScan = 2;
struct CellMeta {
  int16_t n_in;      // input pins I (output pin = I)
  int16_t mode;      // kCellDirect, kCellSipl or kCellScan
  int32_t map_off;   // first map entry
  int32_t leak_off;  // first leakage value
  int32_t axis_off;  // first slew knot: c * n_slew
};
static_assert(sizeof(CellMeta) == 16, "CellMeta is four LDS words");

// Device-memory record of a cell with more than 8 state pins.
struct WideCell {
  int32_t t_first, t_n;   // its table patterns: pat[t_first .. t_first + t_n)
  int32_t l_first, l_n;   // its leakage patterns
  int64_t t_sipl, l_sipl; // kCellSipl: first entry of its per-state item arrays
};

struct WideView {
  const WideCell* cell;   // [n_cells] (entries of kCellDirect cells unused)
  const uint2* pat;       // (care, value) of every pattern
  const uint8_t* sipl;    // per-state item arrays
};

// Item of state s in one of a wide cell's lists: the per-state array, or the
// first pattern whose care pins agree with s (the last pattern of a list has
// care = 0, so the scan always ends on a match).
__device__ __forceinline__ int32_t wide_item(const WideView& W, int cell, int mode, uint32_t s, bool leak) {
  const WideCell& w = W.cell[cell];
  if (mode == kCellSipl) return (int32_t)W.sipl[(leak ? w.l_sipl : w.t_sipl) + (int64_t)s];
  const int32_t first = leak ? w.l_first : w.t_first, n = leak ? w.l_n : w.t_n;
  int32_t k = 0;
#pragma nounroll
  for (; k < n - 1; ++k) {
    const uint2 p = W.pat[first + k];
    if (((s ^ p.y) & p.x) == 0u) break;
  }
  return k;
}

// Library as the kernels see it (device pointers into one ctx-owned buffer).
struct LibView {
  const CellMeta* meta;     // [n_cells]
  const int32_t* map_q;     // [n_map] first quad index of the table
  const float* leak;        // [n_leak]
  const float* load;        // [n_cells * n_load]
  const float* load_inv;    // [n_cells * n_load]
  const float* slew;        // [n_cells * n_slew]
  const float* slew_inv;    // [n_cells * n_slew] 1/(S[i+1]-S[i]) (last unused)
  const float4* quads;      // [n_tables * (n_slew-1) * (n_load-1)]
  int32_t n_cells, n_slew, n_load, n_map, n_leak;
  int32_t lds_words;        // 32-bit words of the LDS image
  int32_t lds_words_ml;     // words of its meta, leakage and load-axis prefix
  int32_t all_pins;         // 1: the state index covers every pin (bit n_in = the output), else the inputs
  WideView wide;            // cells with more than 8 state pins
};

// Mask of the pins the state index covers: the inputs, or every pin.
__device__ __host__ __forceinline__ uint32_t state_mask(int32_t n_in, int32_t all_pins) {
  const int32_t n = n_in + all_pins;
  return n >= 32 ? 0xffffffffu : (1u << n) - 1u;
}

// Prepared gate record (32 bytes), gate-major kernels.
struct GatePrep {
  int32_t cell;
  uint32_t init;      // bit p = initial value of pin p
  int32_t jq;         // load-axis segment of the gate's output load
  float beta;         // load interpolation weight on that segment
  float esw_rise;     // switching energy of an output rise (fJ)
  float esw_fall;     // switching energy of an output fall (fJ)
  float lam;          // leakage scale
  float dbeta_dc;     // 1 / (L[j+1] - L[j])
};
static_assert(sizeof(GatePrep) == 32, "GatePrep is two 16-byte loads");

// Per-call gate record of the packed kernels (8 bytes), indexed by the
// cell-sorted gate index: the load of the gate's output net and its leakage
// scale. The load-axis segment, its weight and the switching energies follow
// from the load and the cell (unit_lut), which keeps the record, gathered
// once per unit, to half a 16-byte vector.
struct GateParam {
  float C;
  float lam;
};
static_assert(sizeof(GateParam) == 8, "GateParam is one 8-byte load");

// Unsigned division of a 32-bit value by an invariant divisor (Granlund and
// Montgomery, "Division by invariant integers using multiplication", PLDI
// 1994, the round-up method for unsigned operands): q = (t1 + ((n - t1) >> s1)) >> s2
// with t1 = mulhi(m, n). Exact for every 32-bit n.
struct Div32 {
  uint32_t m;
  int32_t s1, s2;
};

__device__ __forceinline__ uint32_t div32(uint32_t n, Div32 d) {
  uint32_t t1 = __umulhi(d.m, n);
  return (t1 + ((n - t1) >> d.s1)) >> d.s2;
}

struct BinSpec {
  int64_t D;          // bin width (ps)
  int64_t t_end;
  int64_t n_bins;
  Div32 div;          // division by D, valid when t_end <= 2^32
  int32_t t32;        // 1: times fit 32 bits, use div
  int32_t tile_log2;  // bins per time tile = 2^tile_log2
  int32_t r_bits;     // bits of the in-bin offset r = t - b*D
  int32_t n_tiles;
};

__device__ __forceinline__ int64_t bin_of(int64_t t, const BinSpec& B) {
  if (B.t32) return (int64_t)div32((uint32_t)t, B.div);
  return t / B.D;
}

// LDS image of the library: meta | leak | load | load_inv | map_q | slew |
// slew_inv (words).
struct LdsLib {
  int32_t all_pins;        // as LibView::all_pins
  WideView wide;           // as LibView::wide (device memory)
  const CellMeta* meta;
  const int32_t* map_q;
  const float* leak;
  const float* load;       // [n_cells * n_load] load axes
  const float* load_inv;   // [n_cells * n_load] 1/(L[j+1]-L[j]) (last unused)
  const float* slew;
  const float* slew_inv;
};

__device__ __forceinline__ LdsLib stage_library(const LibView& L, uint32_t* lds) {
  // the image is contiguous in global memory in the same order: copy words
  const uint32_t* src = reinterpret_cast<const uint32_t*>(L.meta);
  for (int w = threadIdx.x; w < L.lds_words; w += blockDim.x) lds[w] = src[w];
  const int32_t nl = L.n_cells * L.n_load;
  LdsLib S;
  S.all_pins = L.all_pins;
  S.wide = L.wide;
  S.meta = reinterpret_cast<const CellMeta*>(lds);
  S.leak = reinterpret_cast<const float*>(lds + 4 * L.n_cells);
  S.load = S.leak + L.n_leak;
  S.load_inv = S.load + nl;
  S.map_q = reinterpret_cast<const int32_t*>(S.load_inv + nl);
  S.slew = reinterpret_cast<const float*>(S.map_q + L.n_map);
  S.slew_inv = S.slew + L.n_cells * L.n_slew;
  return S;
}

// Only the prefix of the image (cell records, leakage values, load axes):
// all the packed kernels read from the library.
__device__ __forceinline__ LdsLib stage_library_ml(const LibView& L, uint32_t* lds) {
  const uint32_t* src = reinterpret_cast<const uint32_t*>(L.meta);
  for (int w = threadIdx.x; w < L.lds_words_ml; w += blockDim.x) lds[w] = src[w];
  const int32_t nl = L.n_cells * L.n_load;
  LdsLib S;
  S.all_pins = L.all_pins;
  S.wide = L.wide;
  S.meta = reinterpret_cast<const CellMeta*>(lds);
  S.leak = reinterpret_cast<const float*>(lds + 4 * L.n_cells);
  S.load = S.leak + L.n_leak;
  S.load_inv = S.load + nl;
  S.map_q = nullptr;
  S.slew = nullptr;
  S.slew_inv = nullptr;
  return S;
}

// Map entry of (state s, new value v) and leakage entry of state s for a
// cell (Lib: LibView or LdsLib; s masked to the cell's state pins).
__device__ __forceinline__ int32_t map_entry_w(const WideView& W, const CellMeta& cm, int cell, uint32_t s,
                                               uint32_t v) {
  const int32_t k = cm.mode == kCellDirect ? (int32_t)s : wide_item(W, cell, cm.mode, s, false);
  return cm.map_off + 2 * k + (int32_t)v;
}
__device__ __forceinline__ int32_t leak_item_w(const WideView& W, const CellMeta& cm, int cell, uint32_t s) {
  return cm.mode == kCellDirect ? (int32_t)s : wide_item(W, cell, cm.mode, s, true);
}
__device__ __forceinline__ int32_t leak_entry_w(const WideView& W, const CellMeta& cm, int cell, uint32_t s) {
  return cm.leak_off + leak_item_w(W, cm, cell, s);
}
template <class Lib>
__device__ __forceinline__ int32_t map_entry(const Lib& L, const CellMeta& cm, int cell, uint32_t s, uint32_t v) {
  return map_entry_w(L.wide, cm, cell, s, v);
}
template <class Lib>
__device__ __forceinline__ int32_t leak_entry(const Lib& L, const CellMeta& cm, int cell, uint32_t s) {
  return leak_entry_w(L.wide, cm, cell, s);
}

// What a unit's gate needs for its events, from its output load C and cell:
// the load-axis segment j = clamp(#knots <= C - 1, 0, n_load - 2), its weight
// beta, d(beta)/dC, and the switching energies of an output rise and fall
// (sw_mode 0: 0.5 C V^2 on both; 1: C V^2 on a rise only). Rounded exactly
// as the gate-major kernels round them.
struct UnitLut {
  uint32_t jq;
  float beta;
  float dbdc;
  float esw_rise, esw_fall;
};

__device__ __forceinline__ UnitLut unit_lut(const LdsLib& L, int32_t n_load, int cell, float C, double v2,
                                            int32_t sw_mode) {
  const float* la = L.load + cell * n_load;
  int j = 0;
  if (n_load == 7) {   // the usual 7 knots: the five interior knots read together
#pragma unroll
    for (int m = 1; m < 6; ++m) j += (la[m] <= C) ? 1 : 0;
  } else {
    for (int m = 1; m < n_load - 1; ++m) j += (la[m] <= C) ? 1 : 0;
  }
  UnitLut u;
  u.jq = (uint32_t)j;
  u.dbdc = L.load_inv[cell * n_load + j];
  u.beta = __fmul_rn(__fsub_rn(C, la[j]), u.dbdc);
  u.esw_rise = (sw_mode == 0) ? (float)(0.5 * (double)C * v2) : (float)((double)C * v2);
  u.esw_fall = sw_mode ? 0.0f : u.esw_rise;
  return u;
}

// Quantised leakage rate of a state (units R = 1e6 * 2^-m nW; rate_scale =
// FP32(2^m * 1e-6)).
__device__ __forceinline__ int32_t qrate(float lam, float leak, float rate_scale) {
  return (int32_t)rintf(__fmul_rn(__fmul_rn(lam, leak), rate_scale));
}

// Energy e (fJ) in units of 2^-40 fJ... generally 2^-m fJ with m = 32 + sh:
// hi = floor(e * 2^sh), lo = (e * 2^sh - hi) * 2^32. Both steps are exact for
// |e| < 2^(31-sh) (the fraction has at most 24 significant bits), so the
// result is e * 2^m truncated toward minus infinity at 2^-m: exact whenever
// e is a multiple of 2^-m, which holds for every FP32 e >= 2^(23-m).
__device__ __forceinline__ int64_t energy_fixed(float e, float two_sh) {
  const float a = __fmul_rn(e, two_sh);
  const float h = floorf(a);
  const float f = __fmul_rn(__fsub_rn(a, h), 4294967296.0f);
  const int32_t hi = (int32_t)h;
  const uint32_t lo = (uint32_t)f;
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint64_t)lo);
}

// Slew segment i = clamp(#knots <= slew - 1, 0, n-2).
__device__ __forceinline__ int slew_seg_index(const float* axis, int n, float slew) {
  int k = 0;
  for (int m = 1; m < n - 1; ++m) k += (axis[m] <= slew) ? 1 : 0;
  return k;
}

// Slew segment i = clamp(#knots <= slew - 1, 0, n-2) and its weight alpha.
__device__ __forceinline__ void slew_segment(const float* axis, const float* inv, int n, float slew, int& i,
                                             float& alpha) {
  int k = 0;
  for (int m = 1; m < n - 1; ++m) k += (axis[m] <= slew) ? 1 : 0;
  i = k;
  alpha = __fmul_rn(__fsub_rn(slew, axis[k]), inv[k]);
}

// Glitch scaling ratio of event e (Sec. 2.4 clock-cycle detection, Eq.
// glitch scaling ratio): the event is a glitch when its pin's previous event
// in the gate's time order lies in the same clock cycle of length clk;
// then r = min(1, (2 pw / (s_prev + s))^2) with pw the time since that event
// and s_prev, s the two slews (FP32), else -1 (a regular event). Searches the
// gate's earlier events (gate-major array, first event gstart) back to the
// start of the cycle.
__device__ __forceinline__ float glitch_ratio(const int64_t* __restrict__ t, const uint8_t* __restrict__ pb,
                                              const float* __restrict__ slew, int64_t gstart, int64_t e, int64_t te,
                                              int pin, float se, int64_t clk) {
  const int64_t c0 = (te / clk) * clk;   // start of the event's clock cycle
  for (int64_t j = e - 1; j >= gstart; --j) {
    const int64_t tj = t[j];
    if (tj < c0) break;
    if ((int)(pb[j] >> 1) == pin) {
      const float q = __fdiv_rn(__fmul_rn(2.0f, (float)(te - tj)), __fadd_rn(slew[j], se));
      return fminf(1.0f, __fmul_rn(q, q));
    }
  }
  return -1.0f;
}

// Bilinear interpolation on a quad (c00, c01, c10, c11) = (T[i][j], T[i][j+1],
// T[i+1][j], T[i+1][j+1]): lerp along the load axis, then along slew.
// Written with explicit roundings so every kernel computes the same bits.
__device__ __forceinline__ float bilerp_quad(float4 q, float alpha, float beta) {
  float a = __fmaf_rn(beta, __fsub_rn(q.y, q.x), q.x);
  float b = __fmaf_rn(beta, __fsub_rn(q.w, q.z), q.z);
  return __fmaf_rn(alpha, __fsub_rn(b, a), a);
}

// d(bilerp)/d(beta)
__device__ __forceinline__ float bilerp_dbeta(float4 q, float alpha) {
  float d0 = __fsub_rn(q.y, q.x);
  float d1 = __fsub_rn(q.w, q.z);
  return __fmaf_rn(alpha, __fsub_rn(d1, d0), d0);
}

// Per-event arithmetic shared by every event-walking kernel.
struct EventOut {
  float e;        // internal + switching energy (fJ)
  int32_t delta;  // leakage step (units R), 0 for output events
  int32_t s;      // input state looked up (before the event's group)
};

// Constants of the fixed-point conversion, shared by all paths.
struct FixArgs {
  float rate_scale;   // FP32(2^m * 1e-6): nW -> R units
  float two_sh;       // 2^(m-32)
};

struct EvView {
  const int64_t* t;
  const uint8_t* pb;
  const float* slew;
  const int64_t* gate_off;
  int64_t n;        // events
  int64_t n_gates;
};

// ---------------------------------------------------------------------------
// gate-major lane-block walker
// ---------------------------------------------------------------------------
// The gate-major event array is cut into lane blocks of kLaneEvents
// consecutive events. One lane walks one block in order, so the gate state is
// a running register (each event toggles one pin: the state is the gate's
// initial bits XOR the parity of the toggles seen so far). A block may hold
// the tail of one gate and many short gates or a slice of one long gate. The
// plan gives every block its first gate and the toggle parity that gate
// carries into the block.
//
// Visitor interface:
//   begin_gate(g, par)  par = parity the gate carries into this block
//   event(k, e, t, pin, v, slew, par_group, par_now)   k = e - first event of the block
//   end_gate(g)
// Events of one gate that share a timestamp form a group; par_group is the
// parity before the group (Algorithm 1 looks up every event of a group with
// the state before it), par_now the parity before this event.
template <class V>
__device__ __forceinline__ void walk_block(int64_t kb, const EvView& E, const uint2* __restrict__ plan, V& vis) {
  const int64_t e0 = kb * kLaneEvents;
  if (e0 >= E.n) return;
  const int nk = (int)min((int64_t)kLaneEvents, E.n - e0);
  int64_t tt[kLaneEvents];
  uint32_t pw[kLaneEvents / 4];
  float sl[kLaneEvents];
  if (nk == kLaneEvents) {
    const longlong2* tp = reinterpret_cast<const longlong2*>(E.t + e0);
#pragma unroll
    for (int k = 0; k < kLaneEvents / 2; ++k) {
      longlong2 v = tp[k];
      tt[2 * k] = v.x;
      tt[2 * k + 1] = v.y;
    }
    const uint4 p4 = *reinterpret_cast<const uint4*>(E.pb + e0);
    pw[0] = p4.x; pw[1] = p4.y; pw[2] = p4.z; pw[3] = p4.w;
    const float4* sp = reinterpret_cast<const float4*>(E.slew + e0);
#pragma unroll
    for (int k = 0; k < kLaneEvents / 4; ++k) {
      float4 v = sp[k];
      sl[4 * k] = v.x; sl[4 * k + 1] = v.y; sl[4 * k + 2] = v.z; sl[4 * k + 3] = v.w;
    }
  } else {
#pragma unroll
    for (int k = 0; k < kLaneEvents / 4; ++k) pw[k] = 0;
#pragma unroll
    for (int k = 0; k < kLaneEvents; ++k) {
      if (k < nk) {
        tt[k] = E.t[e0 + k];
        pw[k >> 2] |= (uint32_t)E.pb[e0 + k] << (8 * (k & 3));
        sl[k] = E.slew[e0 + k];
      } else {
        tt[k] = 0;
        sl[k] = 0.f;
      }
    }
  }
  const uint2 pl = plan[kb];
  int64_t g = (int64_t)pl.x;
  uint32_t par = pl.y;
  int64_t gstart = E.gate_off[g];
  int64_t next_off = E.gate_off[g + 1];
  // A timestamp group may straddle the block start: the group-start parity
  // then excludes the group's earlier events (looked back in memory).
  uint32_t par_gs = par;
  int64_t tprev = INT64_MIN;
  if (e0 > gstart && E.t[e0 - 1] == tt[0]) {
    uint32_t x = 0;
    int64_t j = e0 - 1;
    int guard = 0;
    while (j >= gstart && E.t[j] == tt[0] && guard < 64) {
      x ^= 1u << ((E.pb[j] >> 1) & 31);
      --j;
      ++guard;
    }
    par_gs = par ^ x;
    tprev = tt[0];
  }
  vis.begin_gate(g, par);
#pragma unroll
  for (int k = 0; k < kLaneEvents; ++k) {
    if (k < nk) {
      const int64_t e = e0 + k;
      if (e >= next_off) {
        vis.end_gate(g);
        while (e >= next_off && g < E.n_gates - 1) {
          ++g;
          next_off = E.gate_off[g + 1];
        }
        par = 0;
        tprev = INT64_MIN;
        vis.begin_gate(g, 0u);
      }
      const uint32_t b = (pw[k >> 2] >> (8 * (k & 3))) & 0xffu;
      const int pin = (int)(b >> 1);
      const int v = (int)(b & 1u);
      if (tt[k] != tprev) {
        par_gs = par;
        tprev = tt[k];
      }
      vis.event(k, e, tt[k], pin, v, sl[k], par_gs, par);
      par ^= 1u << (pin & 31);
    }
  }
  vis.end_gate(g);
}

}  // namespace gtp
