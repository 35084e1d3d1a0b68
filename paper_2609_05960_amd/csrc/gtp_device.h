// Device side of the binned power-waveform library (gfx950, wave64).
//
// Data layout in HBM (all struct-of-arrays):
//   events   t int64, pin_bit uint8 ((pin << 1) | new value), slew float,
//            gate-major CSR gate_off int64[G+1] (borrowed from the caller);
//   library  per cell a meta record, the (state, dir) -> table map stored as
//            the table's first quad index, leakage values, slew axis and
//            reciprocal segment widths (all staged in LDS by every kernel),
//            and the tables as "quads": for table T and axis cell (i, j) the
//            four corners (T[i][j], T[i][j+1], T[i+1][j], T[i+1][j+1]) as one
//            16-byte vector, so an interpolation is one 16-byte gather;
//   gates    a 32-byte prepared record per gate, rebuilt on every call from
//            the net loads and leakage scales;
//   bins     int64 fixed-point accumulators X (energy) and S (leakage steps).
//
// Fixed point. Energies are accumulated as integers in units of 2^-k nW*ps
// (1 fJ = 1e6 nW*ps) and leakage rates in units of 2^-k nW, so sums are exact
// and independent of the order of accumulation. The leakage rate of a gate in
// input state s is quantised once, q = rint(lambda * leak[s] * 2^k) (float),
// and every input event adds the step q(after) - q(before): per gate the steps
// telescope exactly, so the rate at any time is exactly the quantised rate of
// the state held.
//
// Leakage in step form (an exact rewrite of the interval rule of Sec. 2.3,
// Eq. leakage energy): with R(t) = sum_g q_g(s_g(t)) the total rate, the
// leakage energy of bin b is  D * R(b*D) + sum over steps d at time t in bin b
// of d * ((b+1)*D - t).  So each input event contributes its step d to S[b]
// and d * ((b+1)*D - t) to X[b]; a prefix sum of S gives R at bin starts.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gtp {

constexpr int kLaneEvents = 16;       // consecutive events per lane block
constexpr int kFwdThreads = 256;      // threads of the event-walking kernels
constexpr int kSubChunk = kLaneEvents * kFwdThreads;  // events per pass of a workgroup
constexpr int kTileThreads = 1024;    // threads of the tile accumulation kernel
constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

// Per-cell record staged in LDS.
struct CellMeta {
  int32_t n_in;      // input pins I (output pin = I)
  int32_t map_off;   // first map entry: entry (s, dir) at map_off + 2*s + dir
  int32_t leak_off;  // first leakage value: state s at leak_off + s
  int32_t axis_off;  // first slew knot: c * n_slew
};

// Library as the kernels see it (device pointers into one ctx-owned buffer).
struct LibView {
  const CellMeta* meta;     // [n_cells]
  const int32_t* map_q;     // [n_map] first quad index of the table
  const float* leak;        // [n_leak]
  const float* slew;        // [n_cells * n_slew]
  const float* slew_inv;    // [n_cells * n_slew] 1/(S[i+1]-S[i]) (last unused)
  const float4* quads;      // [n_tables * (n_slew-1) * (n_load-1)]
  int32_t n_cells, n_slew, n_load, n_map, n_leak;
  int32_t lds_words;        // 32-bit words of the LDS image
};

// Prepared gate record (32 bytes).
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

// LDS image of the library: meta | map_q | leak | slew | slew_inv (words).
struct LdsLib {
  const CellMeta* meta;
  const int32_t* map_q;
  const float* leak;
  const float* slew;
  const float* slew_inv;
};

__device__ __forceinline__ LdsLib stage_library(const LibView& L, uint32_t* lds) {
  // the image is contiguous in global memory in the same order: copy words
  const uint32_t* src = reinterpret_cast<const uint32_t*>(L.meta);
  for (int w = threadIdx.x; w < L.lds_words; w += blockDim.x) lds[w] = src[w];
  LdsLib S;
  S.meta = reinterpret_cast<const CellMeta*>(lds);
  S.map_q = reinterpret_cast<const int32_t*>(lds + 4 * L.n_cells);
  S.leak = reinterpret_cast<const float*>(lds + 4 * L.n_cells + L.n_map);
  S.slew = reinterpret_cast<const float*>(lds + 4 * L.n_cells + L.n_map + L.n_leak);
  S.slew_inv = S.slew + L.n_cells * L.n_slew;
  return S;
}

// Quantised leakage rate of a state (units 2^-k nW).
__device__ __forceinline__ int32_t qrate(float lam, float leak, float scale_k) {
  return (int32_t)rintf(__fmul_rn(__fmul_rn(lam, leak), scale_k));
}

// Slew segment i = clamp(#knots <= slew - 1, 0, n-2) and its weight alpha.
__device__ __forceinline__ void slew_segment(const float* axis, const float* inv, int n, float slew, int& i,
                                             float& alpha) {
  int k = 0;
  for (int m = 1; m < n - 1; ++m) k += (axis[m] <= slew) ? 1 : 0;
  i = k;
  alpha = __fmul_rn(__fsub_rn(slew, axis[k]), inv[k]);
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

// Energy contribution of one event as an integer in units of 2^-k nW*ps.
__device__ __forceinline__ int64_t dyn_fixed(float e_fj, double dyn_scale) {
  return __double2ll_rn((double)e_fj * dyn_scale);
}

// Per-event arithmetic shared by every event-walking kernel.
struct EventOut {
  float e;        // internal + switching energy (fJ)
  int32_t delta;  // leakage step (units 2^-k nW), 0 for output events
  int32_t s;      // input state looked up (before the event's group)
};

}  // namespace gtp
