// Builds the packed, tile-major event layout described in gtp_pack.h.
//
// Steps (all on the caller's stream; the host waits twice, for the number of
// units and the number of groups, which size the arrays, and once at the end
// for the statistics):
//   1. gate order: gates sorted by (cell, octave of the event count largest
//      first, gate) with a device radix sort of 64-bit keys; gate blocks of at most
//      2^gate_block_log2 gates of one cell;
//   2. k_pk_units (count pass): every gate-major lane block of 16 events is
//      walked in order and split into units wherever the gate or the time
//      tile changes; units per block, exclusive scan;
//   3. k_pk_units (emit pass): the same walk writes every unit's sort key
//      (tile, gate block, length class, gate within the block; 32 bits when
//      the fields fit) and its first event, staged in LDS per workgroup;
//   4. device radix sort of the keys with the first events (stable);
//   5. k_pk_bounds: each tile's and each (tile, gate block) region's first
//      unit by binary search over the sorted keys; groups of 64 units per
//      tile, scanned into tile_grp;
//   6. k_pk_group_len: per group its events and longest unit (from the sorted
//      keys), scanned into group offsets; per (tile, gate block) region its
//      events;
//   7. k_pk_fill: one workgroup per tile, one wavefront per group: the unit
//      descriptors, every event's record in the unit-interleaved order, the
//      group's table quad range, and the most events in one bin (LDS
//      histogram of the tile); a unit's carried-in pin values come from the
//      lane-block plan and the pins of its block;
//   8. k_pk_phases + k_pk_phase_copy (the table phases of every tile).
// Temporaries live in a workspace the caller keeps between packs; the pack
// runs once per event set and bin width, its time is reported apart from the
// forward.
#include <hip/hip_runtime.h>
#include <rocprim/device/device_radix_sort.hpp>

#include <algorithm>
#include <cstdio>
#include <vector>

#include "gtp_pack.h"
#include "gtp_scan.h"

namespace gtp {
namespace {

// Sort key of a unit, fields from the most significant: tile, gate block,
// 2^len_bits - length, the gate's index within the block shifted right by
// gin_shift. Within one key the units keep the gate-major order of the walk
// (stable sort); the exact index within the block travels in the unit's first
// event record. The fields are narrowed to 24 bits when the gate index allows
// it (three radix passes), else kept whole in 32 or 64 bits.
struct KeyLayout {
  int32_t len_bits;    // length field (unit lengths 1..2^len_bits)
  int32_t gin_bits;    // width of the gate-index field
  int32_t gin_shift;   // the field holds the gate's index within its block >> gin_shift
  int32_t gb_bits;     // gate-block field
  int32_t tile_bits;
  int32_t time_key;    // 1: the low field holds the top gin_bits bits of the unit's first in-tile bin instead
                       // (the gate index then always travels in the first event record)
};

__host__ __device__ __forceinline__ int key_low(const KeyLayout& L) { return L.len_bits + L.gin_bits; }

template <class K>
__device__ __forceinline__ uint32_t key_len(K key, const KeyLayout& L) {
  return (1u << L.len_bits) - (uint32_t)((key >> L.gin_bits) & (K)((1u << L.len_bits) - 1u));
}
template <class K>
__device__ __forceinline__ uint32_t key_gb(K key, const KeyLayout& L) {
  return (uint32_t)((key >> key_low(L)) & (K)((1ull << L.gb_bits) - 1ull));
}

struct KeySpec {
  KeyLayout L;
  int32_t unit_cap;               // longest unit
};

// Table item of state st and leakage item of state sl of a cell with more
// than 8 state pins (kept out of line: rare, and it would stop the event loop
// of the emit pass from unrolling).
__device__ __noinline__ uint2 wide_items(WideView W, int cell, int mode, uint32_t st, uint32_t sl) {
  return make_uint2((uint32_t)wide_item(W, cell, mode, st, false), (uint32_t)wide_item(W, cell, mode, sl, true));
}

template <class K>
struct UnitArgs {
  EvView ev;
  const uint2* plan;
  const uint4* ginfo;     // per gate: cell, initial pin values, gate block, index within the block
  BinSpec bins;
  KeySpec ks;
  uint32_t* counts;       // count pass: units per lane block
  const uint32_t* base;   // emit pass: first unit of each lane block
  K* keys;                // emit pass: sort key of every unit
  uint32_t* srcs;         // emit pass: gate-major index of every unit's first event
  // emit pass: the workgroup's units staged in LDS (first events as offsets
  // from the workgroup's first event: a workgroup walks kEmitCap events)
  K* lkeys;
  uint16_t* lsrcs;
  uint32_t u0;            // first unit of the workgroup
  int64_t e0;             // first event of the workgroup
  // emit pass: every packed event's record, gate-major (see EvRec)
  LibView lib;
  uint4* rec;
  float* rgl;             // glitch detection on: energy factor of every event, gate-major
  int64_t glitch_clk;
  int32_t* dbg_state;     // optional, gate-major: state before the event's group
  int64_t* dbg_bin;       // optional, gate-major: bin of the event
  int32_t* alpha_span;    // max over events of |1 - alpha| + |alpha| (FP32 bits; positive floats order as ints)
};

// Record of a packed event (16 bytes, gate-major, written by the emit pass
// and gathered unit by unit by the fill): x = the event word (in-tile bin,
// in-bin offset, leakage state after the event), y = the table row at the
// slew segment | output flag | new value, z = the slew weight (FP32 bits),
// w = for a unit's first event, the leakage state before it (its pin values
// for a kCellDirect cell, else its leakage item) | the gate's index within its
// gate block << 16.

template <bool kEmit, class K>
struct UnitVisitor {
  const UnitArgs<K>* A;
  LdsLib L;                // emit pass: the library in LDS
  int64_t kb;
  uint32_t n = 0;          // units closed in this block
  uint32_t gblock = 0;
  uint32_t gin = 0;        // index of the gate within its gate block
  bool open = false;
  int64_t u_src = 0;
  int32_t u_len = 0;
  int64_t u_tile = 0;
  uint32_t u_bl = 0;       // in-tile bin of the unit's first event
  // emit pass: the gate, its cell record and (7-knot slew axes) its knots
  int cell = 0;
  uint32_t init = 0;
  int64_t gstart = 0;
  CellMeta cm;
  uint32_t in_mask = 0;
  float ax[7], ainv[6];
  float span = 1.0f;
  uint4 rbuf[4];           // emit pass: the records of the current 4-event group of the block

  // Records leave in bursts of 4 (64 contiguous bytes per lane), so that
  // every 64-byte piece of the record array is written whole at once.
  __device__ __forceinline__ void put(int k, int64_t e, uint4 r) {   // k: e - the block's first event
    rbuf[k & 3] = r;
    if ((k & 3) == 3) {
      uint4* p = A->rec + (e - 3);
      p[0] = rbuf[0];
      p[1] = rbuf[1];
      p[2] = rbuf[2];
      p[3] = rbuf[3];
    }
  }
  // the last block's final partial group of records (e_end = one past its last event)
  __device__ __forceinline__ void flush(int64_t e_end) {
    const int n = (int)(e_end & 3);
    uint4* p = A->rec + (e_end - n);
#pragma unroll
    for (int i = 0; i < 3; ++i)
      if (i < n) p[i] = rbuf[i];
  }

  __device__ __forceinline__ void close() {
    if (!open) return;
    if (kEmit) {
      const KeyLayout& KL = A->ks.L;
      const int low = key_low(KL);
      const uint32_t field = KL.time_key ? (u_bl >> max(0, A->bins.tile_log2 - KL.gin_bits)) : (gin >> KL.gin_shift);
      const K key = ((K)u_tile << (KL.gb_bits + low)) | ((K)gblock << low) |
                    ((K)((1u << KL.len_bits) - (uint32_t)u_len) << KL.gin_bits) | (K)field;
      const uint32_t i = A->base[kb] + n - A->u0;
      A->lkeys[i] = key;
      A->lsrcs[i] = (uint16_t)(u_src - A->e0);
    }
    ++n;
    open = false;
  }
  __device__ __forceinline__ void begin_gate(int64_t g, uint32_t) {
    open = false;
    if (kEmit) {
      const uint4 gi = A->ginfo[g];
      cell = (int)gi.x;
      init = gi.y;
      gblock = gi.z;
      gin = gi.w;
      if (A->glitch_clk > 0) gstart = A->ev.gate_off[g];
      cm = L.meta[cell];
      in_mask = state_mask(cm.n_in, L.all_pins);
      if (A->lib.n_slew == 7) {
#pragma unroll
        for (int m = 0; m < 7; ++m) ax[m] = L.slew[cm.axis_off + m];
#pragma unroll
        for (int m = 0; m < 6; ++m) ainv[m] = L.slew_inv[cm.axis_off + m];
      }
    }
  }
  __device__ __forceinline__ void end_gate(int64_t) { close(); }
  __device__ __forceinline__ void event(int k, int64_t e, int64_t t, int pin, int v, float slew, uint32_t par_gs,
                                        uint32_t par) {
    const BinSpec& B = A->bins;
    if (t < 0 || t >= B.t_end) {  // outside the window: not packed
      close();
      if (kEmit) put(k, e, make_uint4(0u, 0u, 0u, 0u));
      return;
    }
    const int64_t bin = bin_of(t, B);
    const int64_t tile = bin >> B.tile_log2;
    const bool first = !(open && tile == u_tile && u_len < A->ks.unit_cap);
    if (!first) {
      ++u_len;
    } else {
      close();
      open = true;
      u_src = e;
      u_len = 1;
      u_tile = tile;
      u_bl = (uint32_t)(bin - (tile << B.tile_log2));
    }
    if (kEmit) {
      // Algorithm 1 per event: the table of the input state before the
      // event's timestamp group, the leakage state once its pin has toggled
      const uint32_t before = init ^ par;
      const uint32_t st = (init ^ par_gs) & in_mask;
      uint32_t ti = st, li = (before ^ (1u << (pin & 31))) & in_mask;
      uint32_t lk0 = 0;
      if (cm.mode != kCellDirect) {
        const uint2 w = wide_items(L.wide, cell, cm.mode, st, li);
        ti = w.x;
        li = w.y;
        if (first) lk0 = wide_items(L.wide, cell, cm.mode, 0u, before & in_mask).y;
      } else {
        lk0 = before & 0xffffu;
      }
      int i;
      float al;
      if (A->lib.n_slew == 7) {   // the knots are in registers: the same segment and weight as slew_segment
        i = 0;
#pragma unroll
        for (int m = 1; m < 6; ++m) i += (ax[m] <= slew) ? 1 : 0;
        float a0 = ax[0], iv = ainv[0];
#pragma unroll
        for (int m = 1; m < 6; ++m) {
          a0 = (i == m) ? ax[m] : a0;
          iv = (i == m) ? ainv[m] : iv;
        }
        al = __fmul_rn(__fsub_rn(slew, a0), iv);
      } else {
        slew_segment(L.slew + cm.axis_off, L.slew_inv + cm.axis_off, A->lib.n_slew, slew, i, al);
      }
      const uint32_t q = (uint32_t)(L.map_q[cm.map_off + 2 * (int)ti + v] + i * (A->lib.n_load - 1));
      const uint32_t bl = (uint32_t)(bin - (tile << B.tile_log2));
      const uint32_t rr = (uint32_t)(t - bin * B.D);
      uint4 r;
      r.x = (bl << B.r_bits) | rr | (li << kStateShift);
      r.y = q | ((pin == cm.n_in ? 1u : 0u) << kOutBit) | ((uint32_t)v << 31);
      r.z = __float_as_uint(al);
      r.w = first ? (lk0 | (gin << 16)) : 0u;
      put(k, e, r);
      span = fmaxf(span, fabsf(1.0f - al) + fabsf(al));
      if (A->glitch_clk > 0) {
        const float rg = glitch_ratio(A->ev.t, A->ev.pb, A->ev.slew, gstart, e, t, pin, slew, A->glitch_clk);
        A->rgl[e] = rg > 0.f ? rg : 1.0f;
      }
      if (A->dbg_state) {
        A->dbg_state[e] = (int32_t)st;
        A->dbg_bin[e] = bin;
      }
    }
  }
};

// The parts of the library image the emit pass reads (cell records, then the
// table map and slew axes; the leakage values and load axes are left out).
__host__ __device__ __forceinline__ int32_t emit_lib_words(const LibView& L) {
  return 4 * L.n_cells + L.n_map + 2 * L.n_cells * L.n_slew;
}
__device__ __forceinline__ LdsLib stage_library_emit(const LibView& L, uint32_t* lds) {
  const uint32_t* meta = reinterpret_cast<const uint32_t*>(L.meta);
  const uint32_t* tail = reinterpret_cast<const uint32_t*>(L.map_q);   // map_q | slew | slew_inv
  const int32_t nm = 4 * L.n_cells, nt = L.n_map + 2 * L.n_cells * L.n_slew;
  for (int w = threadIdx.x; w < nm + nt; w += blockDim.x) lds[w] = w < nm ? meta[w] : tail[w - nm];
  LdsLib S;
  S.all_pins = L.all_pins;
  S.wide = L.wide;
  S.meta = reinterpret_cast<const CellMeta*>(lds);
  S.leak = nullptr;
  S.load = nullptr;
  S.load_inv = nullptr;
  S.map_q = reinterpret_cast<const int32_t*>(lds + nm);
  S.slew = reinterpret_cast<const float*>(S.map_q + L.n_map);
  S.slew_inv = S.slew + L.n_cells * L.n_slew;
  return S;
}

// Emit pass: a workgroup's lane blocks own one contiguous run of units
// [base[kb0], base[kb1]) of at most 16 units per lane block; the lanes write
// their units into LDS and the workgroup stores the run with coalesced writes
// (each lane's units would be scattered over the run otherwise). Every lane
// writes its block's event records itself (16 contiguous records per lane,
// in four bursts of four).
constexpr uint32_t kEmitCap = (uint32_t)kLaneEvents * kFwdThreads;
template <bool kEmit, class K>
__global__ void __launch_bounds__(kFwdThreads) k_pk_units(UnitArgs<K> a, int64_t n_blocks) {
  const int64_t kb = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (!kEmit) {
    if (kb >= n_blocks) return;
    UnitVisitor<false, K> vis;
    vis.A = &a;
    vis.kb = kb;
    walk_block(kb, a.ev, a.plan, vis);
    a.counts[kb] = vis.n;
    return;
  }
  extern __shared__ uint64_t lds64[];
  const int64_t kb0 = (int64_t)blockIdx.x * blockDim.x;
  const int64_t kb1 = min(kb0 + (int64_t)blockDim.x, n_blocks);
  const uint32_t u0 = a.base[kb0], n_u = a.base[kb1] - u0;   // n_u <= kEmitCap
  UnitArgs<K> la = a;
  la.lkeys = reinterpret_cast<K*>(lds64);
  la.lsrcs = reinterpret_cast<uint16_t*>(lds64 + kEmitCap * sizeof(K) / 8);
  la.u0 = u0;
  la.e0 = kb0 * kLaneEvents;
  uint32_t* llib = reinterpret_cast<uint32_t*>(lds64 + kEmitCap * (sizeof(K) + 2) / 8);
  UnitVisitor<true, K> vis;
  vis.L = stage_library_emit(a.lib, llib);
  __syncthreads();
  if (kb < n_blocks) {
    vis.A = &la;
    vis.kb = kb;
    walk_block(kb, a.ev, a.plan, vis);
    const int64_t e_end = min((kb + 1) * kLaneEvents, a.ev.n);
    if (e_end & 3) vis.flush(e_end);
  }
  float span = vis.span;
  for (int o = 32; o > 0; o >>= 1) span = fmaxf(span, __shfl_xor(span, o, 64));
  if ((threadIdx.x & 63) == 0) atomicMax(a.alpha_span, __float_as_int(span));
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < n_u; i += blockDim.x) {
    a.keys[u0 + i] = la.lkeys[i];
    a.srcs[u0 + i] = (uint32_t)(la.e0 + la.lsrcs[i]);
  }
}

__global__ void __launch_bounds__(256) k_pk_fill_u32(uint32_t* p, int64_t n, uint32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void __launch_bounds__(256) k_pk_fill_u64(uint64_t* p, int64_t n, uint64_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// First sorted unit at or after a boundary key, by binary search over the
// sorted keys: thread i < n_first gives tile i (i = n_tiles: the end), the
// others the (tile, gate block) regions r = i - n_first (r = n_reg: the end).
// An empty tile or region gets the first unit of the next non-empty one.
template <class K>
__global__ void __launch_bounds__(256) k_pk_bounds(const K* skey, int64_t nu, KeyLayout L, int32_t n_tiles,
                                                   int32_t n_gb, uint32_t* tfirst, uint32_t* rfirst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n_first = (int64_t)n_tiles + 1, n_reg = (int64_t)n_tiles * n_gb;
  if (i >= n_first + n_reg + 1) return;
  const int low = key_low(L), tshift = L.gb_bits + low;
  K target;
  bool end;
  if (i < n_first) {
    end = i == n_tiles;
    target = (K)i << tshift;
  } else {
    const int64_t r = i - n_first;
    end = r == n_reg;
    target = ((K)(r / n_gb) << tshift) | ((K)(r % n_gb) << low);
  }
  int64_t lo = end ? nu : 0, hi = nu;   // the first j with skey[j] >= target
  while (lo < hi) {
    const int64_t m = (lo + hi) >> 1;
    if (skey[m] < target)
      lo = m + 1;
    else
      hi = m;
  }
  if (i < n_first)
    tfirst[i] = (uint32_t)lo;
  else
    rfirst[i - n_first] = (uint32_t)lo;
}

// Groups of every tile: ceil(units / 64).
__global__ void __launch_bounds__(256) k_pk_tile_groups(const uint32_t* tfirst, int32_t n_tiles, uint32_t* gk) {
  const int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k > n_tiles) return;
  gk[k] = (k < n_tiles) ? (tfirst[k + 1] - tfirst[k] + kGroupUnits - 1) / kGroupUnits : 0u;
}

// One workgroup per tile, one wavefront per group: the group's events
// (glen), its longest unit (gmax, the lane steps it costs a wavefront), and the
// events of every (tile, gate block) region (rev, zeroed before; a group spans
// few regions, each summed over its lanes and added once).
constexpr int kGroupLenThreads = 1024;
constexpr int64_t kMaxTileGrid = 1 << 20;   // workgroups of the per-tile builder kernels (a multiple of 8)
template <class K>
__global__ void __launch_bounds__(kGroupLenThreads) k_pk_group_len(const uint32_t* tile_grp, const uint32_t* tfirst, const K* skey,
                                                      KeyLayout L, int32_t n_gb, int64_t* glen, unsigned long long* rev,
                                                      unsigned long long* lane_steps, uint32_t* max_tile_groups,
                                                      int32_t n_tiles) {
  const int lane = (int)(threadIdx.x & 63);
  unsigned long long steps = 0;
  // workgroups stride over the tiles (a grid of one workgroup per tile would
  // exceed the 2^32 work-items of a dispatch for millions of tiles)
  for (int32_t k = blockIdx.x; k < n_tiles; k += gridDim.x) {
    const int64_t g0 = tile_grp[k], g1 = tile_grp[k + 1];
    const int64_t j1 = tfirst[k + 1];
    if (threadIdx.x == 0) atomicMax(max_tile_groups, (uint32_t)(g1 - g0));
    for (int64_t g = g0 + (threadIdx.x >> 6); g < g1; g += blockDim.x >> 6) {
      const int64_t j = tfirst[k] + (g - g0) * kGroupUnits + lane;
      const bool act = j < j1;
      const K key = act ? skey[j] : (K)0;
      const uint32_t len = act ? key_len(key, L) : 0u;
      uint32_t s = len, mx = len;
      for (int o = 32; o > 0; o >>= 1) {
        s += __shfl_xor(s, o, 64);
        mx = max(mx, __shfl_xor(mx, o, 64));
      }
      if (lane == 0) {
        glen[g] = s;
        steps += mx;
      }
      // region events: one pass per distinct region among the active lanes
      const int64_t reg = (int64_t)k * n_gb + (int64_t)key_gb(key, L);
      uint64_t todo = __ballot(act);
      while (todo) {
        const int first = __ffsll((unsigned long long)todo) - 1;
        const int64_t r0 = __shfl(reg, first, 64);
        const bool mine = act && reg == r0;
        const uint64_t m = __ballot(mine);
        uint32_t v = mine ? len : 0u;
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if (lane == first) atomicAdd(&rev[r0], (unsigned long long)v);
        todo &= ~m;
      }
    }
  }
  if (lane == 0 && steps) atomicAdd(lane_steps, steps);
}

struct FillArgs {
  BinSpec bins;
  KeyLayout kl;
  const void* skeys;          // sorted unit keys
  const uint32_t* ssrc;       // gate-major index of each sorted unit's first event
  const int32_t* gb_start;    // [n_gb] first cell-sorted gate of each gate block
  const int32_t* gb_cell;     // [n_gb] cell of each gate block
  const uint4* rec;           // event records (gate-major)
  const float* rgl_g;         // glitch detection on: energy factors (gate-major)
  const uint32_t* tile_grp;
  const uint32_t* tfirst;
  const int64_t* grp_off;
  uint32_t* ev;               // per event its word, table row and slew weight (12 bytes)
  float* rgl;
  uint2* desc;
  int4* gquads;               // optional: quad range of every group's cells (see below)
  const int32_t* cq_lo;       // [n_cells] quad range of each cell's tables
  const int32_t* cq_hi;
  int32_t* max_bin;           // most events in one bin
};

// Item of workgroup w in a launch of n items (n a multiple of 8; items past
// the grid are taken by the workgroups again, w + gridDim.x, ...), so that
// XCD x = w % 8 takes items [x n/8, (x+1) n/8) in launch order.
__device__ __forceinline__ int64_t xcd_item(int64_t w, int64_t n) { return (w % 8) * (n / 8) + w / 8; }

// One workgroup per tile, one wavefront per group of the tile, one lane per
// unit: the unit descriptor (its gate and length from the sort key, the
// leakage state before it and its cell from its first event's record), and
// its event records moved to the unit-interleaved order (the loads of a
// unit's records are issued before any is used: they are scattered over the
// gate-major record array). With gquads set, every group also leaves the
// union of its cells' table quad ranges and its first unit's cell range (lo,
// hi, first lo, first hi; all -1 for an empty group).
constexpr int kFillThreads = 1024;
template <int kS, class K>
__global__ void __launch_bounds__(kFillThreads) k_pk_fill(FillArgs a) {
  // tiles go to XCDs in contiguous ranges (workgroup w runs on XCD w % 8):
  // a gate's records of neighbouring tiles share cache lines, and the
  // workgroups of neighbouring tiles then read them through one L2
  extern __shared__ uint32_t lds[];
  int32_t* hist = reinterpret_cast<int32_t*>(lds);   // events per bin of the tile
  const BinSpec& B = a.bins;
  // workgroups stride over the tiles beyond kMaxTileGrid (a multiple of 8,
  // so a workgroup keeps its XCD's range)
  const int64_t n_items = ((int64_t)B.n_tiles + 7) / 8 * 8;
  for (int64_t it = blockIdx.x; it < n_items; it += gridDim.x) {
    const int32_t k = (int32_t)xcd_item(it, n_items);
    if (k >= B.n_tiles) continue;   // uniform over the workgroup
    __syncthreads();   // the previous tile's histogram has been read
    for (int i = threadIdx.x; i < (1 << B.tile_log2); i += blockDim.x) hist[i] = 0;
    __syncthreads();
    const int lane = (int)(threadIdx.x & 63);
    const int64_t g0 = a.tile_grp[k], g1 = a.tile_grp[k + 1];
    const int64_t jend = a.tfirst[k + 1];
    const K* skeys = static_cast<const K*>(a.skeys);
    const KeyLayout kl = a.kl;
    for (int64_t gi = g0 + (threadIdx.x >> 6); gi < g1; gi += blockDim.x >> 6) {
      const int64_t j = (int64_t)a.tfirst[k] + (gi - g0) * kGroupUnits + lane;
      const bool act = j < jend;
      int len = 0;
      uint32_t gb = 0, gin_k = 0;   // gin_k: the gate-index field (the whole index when not shifted)
      int64_t src = 0;
      if (act) {
        const K key = skeys[j];
        src = (int64_t)a.ssrc[j];
        len = (int)key_len(key, kl);
        gb = key_gb(key, kl);
        gin_k = (uint32_t)(key & (K)((1ull << kl.gin_bits) - 1ull));
      }
      const uint32_t gs0 = act ? (uint32_t)a.gb_start[gb] : 0u;
      const int cell = act ? a.gb_cell[gb] : 0;
      uint4 r[kS];
      float rg[kS];
  #pragma unroll
      for (int kk = 0; kk < kS; ++kk) {
        if (kk < len) {
          r[kk] = a.rec[src + kk];
          if (a.rgl) rg[kk] = a.rgl_g[src + kk];
        }
      }
      // descriptor: the cell-sorted gate | (length - 1) << 28, the leakage state
      // before the unit | cell << 16
      const uint32_t dy = act ? ((r[0].w & 0xffffu) | ((uint32_t)cell << 16)) : 0u;
      const uint32_t gin = (kl.gin_shift || kl.time_key) ? (r[0].w >> 16) : gin_k;
      const uint32_t dx = act ? ((gs0 + gin) | ((uint32_t)(len - 1) << 28)) : 0xffffffffu;
      a.desc[gi * kGroupUnits + lane] = make_uint2(dx, dy);
      if (a.gquads) {
        const uint64_t m = __ballot(act);
        if (m == 0) {
          if (lane == 0) a.gquads[gi] = make_int4(-1, -1, -1, -1);
        } else {
          const int32_t clo = act ? a.cq_lo[cell] : INT32_MAX, chi = act ? a.cq_hi[cell] : INT32_MIN;
          int32_t lo = clo, hi = chi;
          for (int o = 32; o > 0; o >>= 1) {
            lo = min(lo, __shfl_xor(lo, o, 64));
            hi = max(hi, __shfl_xor(hi, o, 64));
          }
          if (lane == __ffsll((unsigned long long)m) - 1) a.gquads[gi] = make_int4(lo, hi, clo, chi);
        }
      }
      // the group's events: per event (in the group's order) its word, row and weight
      const int64_t off0 = a.grp_off[gi];
      uint3* const blk = reinterpret_cast<uint3*>(a.ev) + off0;
      int64_t j0 = 0;   // the group's events before slot kk
  #pragma unroll
      for (int kk = 0; kk < kS; ++kk) {
        const bool on = len > kk;
        const uint64_t m = __ballot(on);
        if (m == 0) break;
        if (on) {
          const uint32_t lo = (uint32_t)m, hi = (uint32_t)(m >> 32);
          const int64_t j = j0 + __builtin_amdgcn_mbcnt_hi(hi, __builtin_amdgcn_mbcnt_lo(lo, 0u));
          atomicAdd(&hist[(r[kk].x & kTimeMask) >> B.r_bits], 1);
          blk[j] = make_uint3(r[kk].x, r[kk].y, r[kk].z);
          if (a.rgl) a.rgl[off0 + j] = rg[kk];
        }
        j0 += __popcll(m);
      }
    }
    __syncthreads();
    int mx = 0;
    for (int i = threadIdx.x; i < (1 << B.tile_log2); i += blockDim.x) mx = max(mx, hist[i]);
    for (int o = 32; o > 0; o >>= 1) mx = max(mx, __shfl_xor(mx, o, 64));
    if (lane == 0 && mx > 0) atomicMax(a.max_bin, mx);
  }
}

// Table phases of one tile (one wavefront per tile): a phase starts at a
// group and grows while the union of its groups' cell table ranges
// [cq_lo, cq_hi) fits the slot (empty groups join the phase they fall in); a
// single group whose cells exceed the slot keeps its first cell's quads
// (full = 0: the other lanes read global memory). The wavefront looks at 64
// groups at a time: the span of the union grows with every group, so the
// phase ends at the first lane whose prefix union exceeds the slot. Phases are
// written at the tile's first group index (a tile has at most as many phases
// as groups) and counted in n_ph; k_pk_phase_copy compacts them.
__global__ void __launch_bounds__(64) k_pk_phases(const int4* gq, const uint32_t* tile_grp, int64_t cap,
                                                  int4* ph_tmp, uint32_t* n_ph, int32_t* all_full) {
  const int32_t k = blockIdx.x;
  const int lane = (int)threadIdx.x;
  const int64_t g0 = tile_grp[k], g1 = tile_grp[k + 1];
  // quad ranges of group e (an inconsistent range counts as an empty group)
  auto quads_of = [&](int64_t e) -> int4 {
    const int4 r = gq[e];
    return (r.x >= 0 && r.y >= r.x && r.z >= r.x && r.w >= r.z && r.w <= r.y) ? r : make_int4(-1, -1, -1, -1);
  };
  uint32_t np = 0;
  int32_t full_all = 1;
  int64_t g = g0;
  while (g < g1) {
    int64_t lo = INT64_MAX, hi = INT64_MIN;   // union of the phase's groups so far
    int64_t e = g;
    for (;;) {
      const int64_t idx = e + lane;
      const int4 r = idx < g1 ? quads_of(idx) : make_int4(-1, -1, -1, -1);
      const bool val = r.x >= 0;
      int64_t plo = val ? (int64_t)r.x : INT64_MAX, phi = val ? (int64_t)r.y : INT64_MIN;
      for (int o = 1; o < 64; o <<= 1) {   // inclusive prefix union over the lanes
        const int64_t ulo = __shfl_up(plo, o, 64), uhi = __shfl_up(phi, o, 64);
        if (lane >= o) {
          plo = min(plo, ulo);
          phi = max(phi, uhi);
        }
      }
      const int64_t nl = min(lo, plo), nh = max(hi, phi);
      const uint64_t brk = __ballot(val && idx > g && nh - nl > cap);
      if (brk) {
        const int f = __ffsll((unsigned long long)brk) - 1;   // > 0 unless the phase started in an earlier chunk
        const int64_t bl = __shfl(nl, max(f - 1, 0), 64), bh = __shfl(nh, max(f - 1, 0), 64);
        if (f > 0) {
          lo = bl;
          hi = bh;
        }
        e += f;
        break;
      }
      lo = __shfl(nl, 63, 64);
      hi = __shfl(nh, 63, 64);
      e += 64;
      if (e >= g1) {
        e = g1;
        break;
      }
    }
    if (lo == INT64_MAX) {  // only empty groups: nothing to stage
      lo = 0;
      hi = 0;
    }
    int32_t full = 1;
    if (hi - lo > cap) {  // group g alone exceeds the slot (so it is not empty)
      const int4 r = quads_of(g);
      lo = r.x >= 0 ? r.z : 0;
      hi = r.x >= 0 ? min((int64_t)r.w, lo + cap) : 0;
      full = 0;
      full_all = 0;
    }
    if (lane == 0) ph_tmp[g0 + np] = make_int4((int32_t)(e - g0), (int32_t)lo, (int32_t)(hi - lo), full);
    ++np;
    g = e;
  }
  if (lane == 0) {
    n_ph[k] = np;
    if (!full_all) atomicAnd(all_full, 0);
  }
}

__global__ void __launch_bounds__(256) k_pk_phase_copy(const int4* ph_tmp, const uint32_t* tile_grp,
                                                       const uint32_t* ph_off, int32_t n_tiles, int4* phases) {
  const int32_t k = blockIdx.x;
  const uint32_t n = ph_off[k + 1] - ph_off[k];
  for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) phases[ph_off[k] + i] = ph_tmp[tile_grp[k] + i];
}

// Output nets and initial pin values in cell-sorted gate order (the per-call
// gate records then read them contiguously).
// Also the per-gate record of the unit walk (cell, initial pin values, gate
// block, index within the block).
__global__ void __launch_bounds__(256) k_pk_gate_sorted(const int32_t* gperm, const int32_t* gcell,
                                                        const int32_t* gate_out, const uint32_t* gate_init,
                                                        const int32_t* cell_start, const int32_t* gb_base,
                                                        int32_t gb_log2, int64_t n_gates, int32_t* gout,
                                                        uint32_t* ginit, uint4* ginfo) {
  const int64_t gs = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gs >= n_gates) return;
  const int32_t g = gperm[gs];
  const int32_t c = gcell[gs];
  const uint32_t init = gate_init[g];
  gout[gs] = gate_out[g];
  ginit[gs] = init;
  const int32_t in_cell = (int32_t)gs - cell_start[c];
  ginfo[g] = make_uint4((uint32_t)c, init, (uint32_t)(gb_base[c] + (in_cell >> gb_log2)),
                        (uint32_t)in_cell & ((1u << gb_log2) - 1u));
}

constexpr int kGateCellShift = 35;   // gate key: cell | 64 - octave (7 bits) | gate (28 bits)

// Sort key of gate g for the cell-sorted gate order: cell, then the octave
// of its weight (its event count unless weights are given), largest first,
// then the gate index (n_cells < 2^16, gates < 2^28). Busy gates come first,
// so the long units of a tile lie in a few cache lines of gate records; gates
// of one octave keep the caller's order, which is the order the emit pass
// meets them in, so units that tie on a narrowed sort key are already in gate
// order (a wavefront's gate records then span fewer lines).
__global__ void __launch_bounds__(256) k_pk_gate_keys(const int32_t* gate_cell, const int64_t* gate_off,
                                                      const int64_t* weight, int64_t n_gates, uint64_t* keys) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n_gates) return;
  const int64_t w = weight ? weight[g] : gate_off[g + 1] - gate_off[g];
  const int oct = w > 0 ? 64 - __clzll((unsigned long long)w) : 0;   // bit length, 0..63
  keys[g] = ((uint64_t)(uint32_t)gate_cell[g] << kGateCellShift) | ((uint64_t)(64 - oct) << 28) | (uint64_t)g;
}

// The sorted keys as the permutation (sorted index -> gate) and each sorted
// gate's cell.
__global__ void __launch_bounds__(256) k_pk_gate_order(const uint64_t* skeys, int64_t n_gates, int32_t* perm,
                                                       int32_t* pcell) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n_gates) return;
  const uint64_t k = skeys[r];
  perm[r] = (int32_t)(k & ((1u << 28) - 1u));
  pcell[r] = (int32_t)(k >> kGateCellShift);
}

int ceil_log2_u64(uint64_t x) {
  int l = 0;
  while ((1ull << l) < x) ++l;
  return l;
}

// Bump allocator over the caller's workspace (256-byte aligned pieces).
struct Bump {
  char* base;
  size_t cap, used = 0;
  template <class T>
  T* take(size_t count) {
    const size_t bytes = (std::max<size_t>(count, 1) * sizeof(T) + 255) & ~(size_t)255;
    if (used + bytes > cap) return nullptr;
    T* p = reinterpret_cast<T*>(base + used);
    used += bytes;
    return p;
  }
};

size_t align256(size_t b) { return (std::max<size_t>(b, 1) + 255) & ~(size_t)255; }

// Exclusive scan (add) of n items with the three-pass scan kernels; sums
// holds ceil(n / kScanTile) items.
template <class T>
void scan_add(const T* in, T* out, T* sums, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  const int64_t nt = (n + kScanTile - 1) / kScanTile;
  hipLaunchKernelGGL((k_scan_tiles<T, OpAdd>), dim3((unsigned)nt), dim3(kScanThreads), 0, s, in, out, sums, n, (T)0,
                     OpAdd());
  if (nt > 1) {
    hipLaunchKernelGGL((k_scan_sums<T, OpAdd>), dim3(1), dim3(kScanThreads), 0, s, sums, nt, (T)0, OpAdd());
    hipLaunchKernelGGL((k_scan_add<T, OpAdd>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, out,
                       (const T*)sums, n, OpAdd());
  }
}

int64_t scan_sums_items(int64_t n) { return (n + kScanTile - 1) / kScanTile + 1; }

// Key-type dispatch of the unit steps.
template <class K>
hipError_t launch_emit(const UnitArgs<uint32_t>& u, void* keys, uint32_t* srcs, int64_t n_blocks, unsigned grid,
                       hipStream_t s) {
  UnitArgs<K> a;
  a.ev = u.ev;
  a.plan = u.plan;
  a.ginfo = u.ginfo;
  a.bins = u.bins;
  a.ks = u.ks;
  a.counts = u.counts;
  a.base = u.base;
  a.keys = static_cast<K*>(keys);
  a.srcs = srcs;
  a.lkeys = nullptr;
  a.lsrcs = nullptr;
  a.u0 = 0;
  a.lib = u.lib;
  a.rec = u.rec;
  a.rgl = u.rgl;
  a.glitch_clk = u.glitch_clk;
  a.dbg_state = u.dbg_state;
  a.dbg_bin = u.dbg_bin;
  a.alpha_span = u.alpha_span;
  // staged keys and first events, then the library image
  const size_t lds = (size_t)kEmitCap * (sizeof(K) + sizeof(uint16_t)) + (size_t)emit_lib_words(u.lib) * 4;
  const hipError_t e =
      hipFuncSetAttribute((const void*)k_pk_units<true, K>, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_pk_units<true, K>), dim3(grid), dim3(kFwdThreads), lds, s, a, n_blocks);
  return hipSuccess;
}

// Stable radix sort of the unit keys with their first events (tmp null:
// the temporary size only). Keys of up to 24 bits take three passes of 8-bit
// digits; wider 32-bit keys take 10-bit digits (the widest a 1024-thread
// workgroup ranks), so that 30 bits still sort in three passes: on 10^9
// events that is one pass less than four 8-bit passes (about 0.5 ms of a
// 29 ms layout build), while three 10-bit passes over a 24-bit key are slower
// than three 8-bit ones.
hipError_t sort_units(bool key64, void* tmp, size_t& tb, void* keys, void* skeys, uint32_t* srcs, uint32_t* ssrc,
                      int64_t n, int bits, hipStream_t s) {
  if (key64)
    return rocprim::radix_sort_pairs(tmp, tb, static_cast<uint64_t*>(keys), static_cast<uint64_t*>(skeys), srcs, ssrc,
                                     n, 0, bits, s);
  if (bits > 24) {
    using cfg = rocprim::radix_sort_config<
        rocprim::default_config, rocprim::default_config,
        rocprim::radix_sort_onesweep_config<rocprim::kernel_config<1024, 16>, rocprim::kernel_config<1024, 16>, 10,
                                            rocprim::block_radix_rank_algorithm::match>>;
    return rocprim::radix_sort_pairs<cfg>(tmp, tb, static_cast<uint32_t*>(keys), static_cast<uint32_t*>(skeys), srcs,
                                          ssrc, n, 0, bits, s);
  }
  return rocprim::radix_sort_pairs(tmp, tb, static_cast<uint32_t*>(keys), static_cast<uint32_t*>(skeys), srcs, ssrc,
                                   n, 0, bits, s);
}

hipError_t launch_fill(bool short_units, bool key64, const FillArgs& fa, unsigned grid, size_t lds, hipStream_t s) {
  const void* fn = short_units ? (key64 ? (const void*)k_pk_fill<8, uint64_t> : (const void*)k_pk_fill<8, uint32_t>)
                               : (key64 ? (const void*)k_pk_fill<16, uint64_t> : (const void*)k_pk_fill<16, uint32_t>);
  const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  if (e != hipSuccess) return e;
  if (short_units) {
    if (key64)
      hipLaunchKernelGGL((k_pk_fill<8, uint64_t>), dim3(grid), dim3(kFillThreads), lds, s, fa);
    else
      hipLaunchKernelGGL((k_pk_fill<8, uint32_t>), dim3(grid), dim3(kFillThreads), lds, s, fa);
  } else {
    if (key64)
      hipLaunchKernelGGL((k_pk_fill<16, uint64_t>), dim3(grid), dim3(kFillThreads), lds, s, fa);
    else
      hipLaunchKernelGGL((k_pk_fill<16, uint32_t>), dim3(grid), dim3(kFillThreads), lds, s, fa);
  }
  return hipSuccess;
}

}  // namespace

void pack_free(PackOut* o) {
  void* ps[] = {o->ev,   o->rgl,   o->desc,  o->grp_off, o->tile_grp, o->gperm, o->gcell,
                o->gout, o->ginit, o->reg_first, o->tfirst, o->phases, o->ph_off};
  for (void* p : ps) {
    const char* q = static_cast<const char*>(p);
    if (p && !(o->arena_lo && q >= o->arena_lo && q < o->arena_lo + o->arena_len)) (void)hipFree(p);
  }
  *o = PackOut();
}

hipError_t pack_events(const PackIn& in, PackOut* out, char* err, size_t err_len) {
  PackOut o;
  hipError_t st = hipSuccess;
  const hipStream_t s = in.stream;
  const int64_t G = in.ev.n_gates, N = in.ev.n;
  const int32_t n_cells = (int32_t)in.n_in.size();
  const BinSpec& B = in.bins;
  const int32_t n_tiles = B.n_tiles;
  int64_t held = 0;
  Workspace* ws = in.ws;         // gate order and unit counts
  Workspace* ws2b = in.ws + 1;   // units, sort, offsets, phases

#define PK(call)                                                                   \
  do {                                                                             \
    st = (call);                                                                   \
    if (st != hipSuccess) {                                                        \
      snprintf(err, err_len, "pack: %s: %s", #call, hipGetErrorString(st));        \
      goto fail;                                                                   \
    }                                                                              \
  } while (0)
#define PKLAUNCH(name)                                                             \
  do {                                                                             \
    st = hipGetLastError();                                                        \
    if (st != hipSuccess) {                                                        \
      snprintf(err, err_len, "pack: launch of %s: %s", name, hipGetErrorString(st)); \
      goto fail;                                                                   \
    }                                                                              \
  } while (0)

  // owned output arrays: carved from the arena while it has room, else
  // allocated (and freed by pack_free)
  size_t arena_used = 0;
  if (in.arena && in.arena->p) {
    o.arena_lo = static_cast<char*>(in.arena->p);
    o.arena_len = in.arena->bytes;
  }
  auto own = [&](size_t bytes, hipError_t& e) -> void* {
    void* p = nullptr;
    bytes = align256(std::max<size_t>(bytes, 256));
    o.need_bytes += bytes;
    if (o.arena_lo && arena_used + bytes <= o.arena_len) {
      p = o.arena_lo + arena_used;
      arena_used += bytes;
      e = hipSuccess;
      return p;
    }
    e = hipMalloc(&p, bytes);
    if (e == hipSuccess) held += (int64_t)bytes;
    return p;
  };
  // grows a workspace to at least `bytes` (after the stream is idle: no
  // earlier use of the old buffer is pending)
  auto reserve = [&](Workspace* w, size_t bytes) -> hipError_t {
    if (w->bytes >= bytes) return hipSuccess;
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    if (w->p) (void)hipFree(w->p);
    w->p = nullptr;
    w->bytes = 0;
    e = hipMalloc(&w->p, bytes);
    if (e != hipSuccess) {
      w->p = nullptr;
      return e;
    }
    w->bytes = bytes;
    return hipSuccess;
  };

  {
    // ---- 1. gate order ------------------------------------------------------
    std::vector<int32_t> cnt(n_cells + 1, 0), cell_start(n_cells, 0), gb_base(n_cells, 0);
    for (int64_t g = 0; g < G; ++g) cnt[in.h_gate_cell[g]]++;
    int32_t acc = 0, gbacc = 0;
    for (int32_t c = 0; c < n_cells; ++c) {
      cell_start[c] = acc;
      gb_base[c] = gbacc;
      acc += cnt[c];
      gbacc += (cnt[c] + (1 << in.gate_block_log2) - 1) >> in.gate_block_log2;
    }
    const int32_t n_gb = std::max(gbacc, 1);
    o.n_gb = n_gb;
    o.gb_log2 = in.gate_block_log2;
    o.h_gb_start.assign((size_t)n_gb + 1, (int32_t)G);
    o.h_gb_cell.assign((size_t)n_gb, 0);
    for (int32_t c = 0; c < n_cells; ++c)
      for (int32_t b = 0; gb_base[c] + b < (c + 1 < n_cells ? gb_base[c + 1] : gbacc); ++b) {
        o.h_gb_start[gb_base[c] + b] = cell_start[c] + (b << in.gate_block_log2);
        o.h_gb_cell[gb_base[c] + b] = c;
      }
    if (n_cells >= (1 << 16) || G >= (1ll << 28)) {
      snprintf(err, err_len, "pack: %d cells, %lld gates", n_cells, (long long)G);
      return hipErrorInvalidValue;
    }
    KeyLayout kl;
    kl.len_bits = ceil_log2_u64((uint64_t)std::max(in.unit_events, 1));
    kl.gb_bits = ceil_log2_u64((uint64_t)n_gb);
    kl.tile_bits = std::max(1, ceil_log2_u64((uint64_t)n_tiles));
    {
      // the gate-index field takes what is left of 24 bits, else of 30 (three
      // passes either way, see sort_units), else of 32 (or all 64: every
      // field whole); the record carries the index in 16 bits, so larger gate
      // blocks keep it whole in the key
      const int head = kl.tile_bits + kl.gb_bits + kl.len_bits;
      const int room = head <= 24 ? 24 - head : (head <= 30 ? 30 - head : (head <= 32 ? 32 - head : in.gate_block_log2));
      kl.gin_bits = in.gate_block_log2 > 16 ? in.gate_block_log2 : std::min(room, in.gate_block_log2);
      kl.gin_shift = in.gate_block_log2 - kl.gin_bits;
      kl.time_key = (in.time_order && in.gate_block_log2 <= 16) ? 1 : 0;
      if (kl.time_key) {   // the in-tile bin, whole or its top bits, in 30 bits when they hold the rest
        const int tb = in.bins.tile_log2;
        kl.gin_bits = head + tb <= 30 ? tb : (head <= 30 ? 30 - head : std::max(0, std::min(tb, 64 - head)));
      }
    }
    const int gb_bits = kl.gb_bits;
    const int low = key_low(kl);   // length and gate-index fields
    const int key_bits = kl.tile_bits + gb_bits + low;
    if (key_bits > 64) {
      snprintf(err, err_len, "pack: sort key of %d bits", key_bits);
      return hipErrorInvalidValue;
    }
    const bool key64 = key_bits > 32;
    const size_t ksz = key64 ? 8 : 4;
    if (N >= (int64_t)UINT32_MAX) {   // units name their first event with 32 bits
      snprintf(err, err_len, "pack: %lld events in one layout (at most 2^32 - 1; use time windows)", (long long)N);
      return hipErrorInvalidValue;
    }
    const int64_t n_blocks = (N + kLaneEvents - 1) / kLaneEvents;
    hipError_t e2;
    o.gperm = (int32_t*)own((size_t)G * 4, e2);
    PK(e2);
    o.gcell = (int32_t*)own((size_t)G * 4, e2);
    PK(e2);
    o.gout = (int32_t*)own((size_t)G * 4, e2);
    PK(e2);
    o.ginit = (uint32_t*)own((size_t)G * 4, e2);
    PK(e2);

    // workspace, phase 1: gate sort and unit counts (sized before the unit count is known)
    size_t gsort_tmp = 0;
    if (G > 0)
      PK(rocprim::radix_sort_keys(nullptr, gsort_tmp, (uint64_t*)nullptr, (uint64_t*)nullptr, (int64_t)G, 0,
                                  kGateCellShift + std::max(1, ceil_log2_u64((uint64_t)n_cells)), s));
    const size_t ws1 = 2 * align256((size_t)n_cells * 4) + 3 * align256((size_t)G * 8) +
                       align256(gsort_tmp) + 2 * align256((size_t)(n_blocks + 1) * 4) +
                       align256((size_t)scan_sums_items(n_blocks + 1) * 4) + align256(64) +
                       2 * align256((size_t)n_gb * 4) + align256((size_t)G * sizeof(uint4));
    PK(reserve(ws, ws1));
    Bump wb{(char*)ws->p, ws->bytes};
    int32_t* d_cs = wb.take<int32_t>((size_t)n_cells);
    int32_t* d_gbb = wb.take<int32_t>((size_t)n_cells);
    uint32_t* counts = wb.take<uint32_t>((size_t)n_blocks + 1);
    uint32_t* ubase = wb.take<uint32_t>((size_t)n_blocks + 1);
    uint32_t* usums = wb.take<uint32_t>((size_t)scan_sums_items(n_blocks + 1));
    uint32_t* d_nu = wb.take<uint32_t>(16);
    int32_t* d_gbs = wb.take<int32_t>((size_t)n_gb);
    int32_t* d_gbc = wb.take<int32_t>((size_t)n_gb);
    uint4* ginfo = wb.take<uint4>((size_t)G);
    PK(hipMemcpyAsync(d_cs, cell_start.data(), (size_t)n_cells * 4, hipMemcpyHostToDevice, s));
    PK(hipMemcpyAsync(d_gbb, gb_base.data(), (size_t)n_cells * 4, hipMemcpyHostToDevice, s));
    PK(hipMemcpyAsync(d_gbs, o.h_gb_start.data(), (size_t)n_gb * 4, hipMemcpyHostToDevice, s));
    PK(hipMemcpyAsync(d_gbc, o.h_gb_cell.data(), (size_t)n_gb * 4, hipMemcpyHostToDevice, s));
    if (G > 0) {
      uint64_t* gk = wb.take<uint64_t>((size_t)G);
      uint64_t* gks = wb.take<uint64_t>((size_t)G);
      int64_t* d_wt = wb.take<int64_t>((size_t)G);
      void* tsort = wb.take<char>(gsort_tmp);
      const bool wt = (int64_t)in.gate_weight.size() == G;
      if (wt) PK(hipMemcpyAsync(d_wt, in.gate_weight.data(), (size_t)G * 8, hipMemcpyHostToDevice, s));
      const dim3 gg((unsigned)((G + 255) / 256));
      hipLaunchKernelGGL(k_pk_gate_keys, gg, dim3(256), 0, s, in.gate_cell, in.ev.gate_off,
                         wt ? (const int64_t*)d_wt : nullptr, (int64_t)G, gk);
      PKLAUNCH("k_pk_gate_keys");
      size_t tb = gsort_tmp;
      PK(rocprim::radix_sort_keys(tsort, tb, gk, gks, (int64_t)G, 0,
                                  kGateCellShift + std::max(1, ceil_log2_u64((uint64_t)n_cells)), s));
      hipLaunchKernelGGL(k_pk_gate_order, gg, dim3(256), 0, s, gks, (int64_t)G, o.gperm, o.gcell);
      PKLAUNCH("k_pk_gate_order");
      hipLaunchKernelGGL(k_pk_gate_sorted, gg, dim3(256), 0, s, o.gperm, o.gcell, in.gate_out, in.gate_init,
                         (const int32_t*)d_cs, (const int32_t*)d_gbb, (int32_t)in.gate_block_log2, (int64_t)G, o.gout,
                         o.ginit, ginfo);
      PKLAUNCH("k_pk_gate_sorted");
    }

    // ---- 2. unit counts ----------------------------------------------------
    UnitArgs<uint32_t> ua;
    ua.ev = in.ev;
    ua.plan = in.plan_blk;
    ua.ginfo = ginfo;
    ua.bins = B;
    ua.ks.L = kl;
    ua.ks.unit_cap = in.unit_events;
    ua.counts = counts;
    ua.base = ubase;
    ua.keys = nullptr;
    ua.srcs = nullptr;
    ua.lkeys = nullptr;
    ua.lsrcs = nullptr;
    ua.u0 = 0;
    ua.lib = LibView();
    ua.rec = nullptr;
    ua.rgl = nullptr;
    ua.glitch_clk = 0;
    ua.dbg_state = nullptr;
    ua.dbg_bin = nullptr;
    ua.alpha_span = nullptr;
    int64_t NU = 0;
    if (n_blocks > 0) {
      const unsigned gridb = (unsigned)((n_blocks + kFwdThreads - 1) / kFwdThreads);
      hipLaunchKernelGGL((k_pk_units<false, uint32_t>), dim3(gridb), dim3(kFwdThreads), 0, s, ua, n_blocks);
      PKLAUNCH("k_pk_units<count>");
      hipLaunchKernelGGL(k_pk_fill_u32, dim3(1), dim3(256), 0, s, counts + n_blocks, (int64_t)1, 0u);
      PKLAUNCH("k_pk_fill_u32");
      scan_add<uint32_t>(counts, ubase, usums, n_blocks + 1, s);
      PKLAUNCH("scan of unit counts");
      uint32_t tot = 0;
      PK(hipMemcpyAsync(&tot, ubase + n_blocks, 4, hipMemcpyDeviceToHost, s));
      PK(hipStreamSynchronize(s));
      NU = tot;
    }
    o.n_units = NU;
    const int64_t n_reg = (int64_t)n_tiles * n_gb;

    // workspace, phase 2 (a second buffer: the first one's pieces stay in use)
    size_t usort_tmp = 0;
    if (NU > 0) PK(sort_units(key64, nullptr, usort_tmp, nullptr, nullptr, nullptr, nullptr, NU, key_bits, s));
    const int64_t ng_max = NU / kGroupUnits + n_tiles + 1;   // groups per tile: ceil(units / 64)
    const size_t ws2 = 2 * align256((size_t)NU * ksz) + 2 * align256((size_t)NU * 4) + align256(usort_tmp) +
                       align256((size_t)(n_tiles + 1) * 4) + align256((size_t)scan_sums_items(n_tiles + 1) * 4) +
                       align256((size_t)(ng_max + 1) * 8) + align256((size_t)scan_sums_items(ng_max + 1) * 8) +
                       align256((size_t)std::max<int64_t>(n_reg, 1) * 8) +
                       2 * align256((size_t)ng_max * sizeof(int4)) +
                       align256((size_t)(n_tiles + 1) * 4) + align256((size_t)scan_sums_items(n_tiles + 1) * 4) +
                       align256((size_t)n_cells * 8) + align256((size_t)N * sizeof(uint4)) +
                       (in.glitch_clk > 0 ? align256((size_t)N * 4) : 0) + 4096;
    PK(reserve(ws2b, ws2));
    Bump wc{(char*)ws2b->p, ws2b->bytes};
    void* keys = wc.take<char>((size_t)NU * ksz);
    void* skeys = wc.take<char>((size_t)NU * ksz);
    uint32_t* srcs = wc.take<uint32_t>((size_t)NU);
    uint32_t* ssrc = wc.take<uint32_t>((size_t)NU);
    void* tsortu = wc.take<char>(usort_tmp);
    uint32_t* gk = wc.take<uint32_t>((size_t)n_tiles + 1);
    uint32_t* tsums = wc.take<uint32_t>((size_t)scan_sums_items(n_tiles + 1));
    int64_t* glen = wc.take<int64_t>((size_t)ng_max + 1);
    int64_t* gsums = wc.take<int64_t>((size_t)scan_sums_items(ng_max + 1));
    int64_t* rev = wc.take<int64_t>((size_t)std::max<int64_t>(n_reg, 1));
    int4* gquads = wc.take<int4>((size_t)ng_max);
    int4* ph_tmp = wc.take<int4>((size_t)ng_max);
    uint32_t* nph = wc.take<uint32_t>((size_t)n_tiles + 1);
    uint32_t* psums = wc.take<uint32_t>((size_t)scan_sums_items(n_tiles + 1));
    int32_t* d_cq = wc.take<int32_t>(2 * (size_t)n_cells);
    uint4* rec = wc.take<uint4>((size_t)N);
    float* rgl_g = in.glitch_clk > 0 ? wc.take<float>((size_t)N) : nullptr;
    if (!d_cq || !rec || (in.glitch_clk > 0 && !rgl_g)) {
      snprintf(err, err_len, "pack: workspace of %zu bytes too small", ws2b->bytes);
      st = hipErrorOutOfMemory;
      goto fail;
    }
    // d_nu[0..]: alpha span bits, max events per bin, lane steps (u64 at 2..3),
    // max tile groups, all-phases-full flag
    {
      const int32_t init[8] = {__builtin_bit_cast(int32_t, 1.0f), 0, 0, 0, 0, 1, 0, 0};
      PK(hipMemcpyAsync(d_nu, init, sizeof init, hipMemcpyHostToDevice, s));
    }
    if (NU > 0) {
      // ---- 3. units --------------------------------------------------------
      const unsigned gridb = (unsigned)((n_blocks + kFwdThreads - 1) / kFwdThreads);
      ua.lib = in.lib;
      ua.rec = rec;
      ua.rgl = rgl_g;
      ua.glitch_clk = in.glitch_clk;
      ua.dbg_state = in.dbg_state;
      ua.dbg_bin = in.dbg_bin;
      ua.alpha_span = (int32_t*)d_nu;
      PK(key64 ? launch_emit<uint64_t>(ua, keys, srcs, n_blocks, gridb, s)
               : launch_emit<uint32_t>(ua, keys, srcs, n_blocks, gridb, s));
      PKLAUNCH("k_pk_units<emit>");
      // ---- 4. sort --------------------------------------------------------
      size_t tb = usort_tmp;
      PK(sort_units(key64, tsortu, tb, keys, skeys, srcs, ssrc, NU, key_bits, s));
    }
    // ---- 5. tiles and groups -------------------------------------------
    o.tfirst = (uint32_t*)own((size_t)(n_tiles + 1) * 4, e2);
    PK(e2);
    o.tile_grp = (int32_t*)own((size_t)(n_tiles + 1) * 4, e2);
    PK(e2);
    o.reg_first = (uint32_t*)own((size_t)(n_reg + 1) * 4, e2);
    PK(e2);
    {
      const int64_t nb = (int64_t)n_tiles + 1 + n_reg + 1;
      const dim3 gbd((unsigned)((nb + 255) / 256));
      if (key64)
        hipLaunchKernelGGL(k_pk_bounds<uint64_t>, gbd, dim3(256), 0, s, (const uint64_t*)skeys, NU, kl, n_tiles, n_gb,
                           o.tfirst, o.reg_first);
      else
        hipLaunchKernelGGL(k_pk_bounds<uint32_t>, gbd, dim3(256), 0, s, (const uint32_t*)skeys, NU, kl, n_tiles, n_gb,
                           o.tfirst, o.reg_first);
      PKLAUNCH("k_pk_bounds");
    }
    hipLaunchKernelGGL(k_pk_tile_groups, dim3((unsigned)((n_tiles + 1 + 255) / 256)), dim3(256), 0, s,
                       (const uint32_t*)o.tfirst, n_tiles, gk);
    PKLAUNCH("k_pk_tile_groups");
    scan_add<uint32_t>(gk, (uint32_t*)o.tile_grp, tsums, n_tiles + 1, s);
    PKLAUNCH("scan of tile groups");
    uint32_t ngu = 0;
    PK(hipMemcpyAsync(&ngu, o.tile_grp + n_tiles, 4, hipMemcpyDeviceToHost, s));
    PK(hipStreamSynchronize(s));
    const int64_t ng = ngu;
    if (ng >= (int64_t)INT32_MAX || ng > ng_max) {
      snprintf(err, err_len, "pack: %lld groups", (long long)ng);
      st = hipErrorInvalidValue;
      goto fail;
    }
    o.n_groups = ng;
    // ---- 6. group and unit lengths, offsets, regions ------------------------
    o.grp_off = (int64_t*)own((size_t)(ng + 1) * 8, e2);
    PK(e2);
    hipLaunchKernelGGL(k_pk_fill_u64, dim3(1), dim3(256), 0, s, (uint64_t*)(glen + ng), (int64_t)1, (uint64_t)0);
    PKLAUNCH("k_pk_fill_u64");
    if (n_reg > 0) {
      hipLaunchKernelGGL(k_pk_fill_u64, dim3((unsigned)((n_reg + 255) / 256)), dim3(256), 0, s, (uint64_t*)rev, n_reg,
                         (uint64_t)0);
      PKLAUNCH("k_pk_fill_u64");
    }
    // workgroups of the per-tile kernels: one per tile up to kMaxTileGrid (a
    // multiple of 8), striding beyond
    const unsigned grid_tiles = (unsigned)std::min<int64_t>(((int64_t)n_tiles + 7) / 8 * 8, kMaxTileGrid);
    if (key64)
      hipLaunchKernelGGL(k_pk_group_len<uint64_t>, dim3(grid_tiles), dim3(kGroupLenThreads), 0, s,
                         (const uint32_t*)o.tile_grp, (const uint32_t*)o.tfirst, (const uint64_t*)skeys, kl, n_gb,
                         glen, (unsigned long long*)rev, (unsigned long long*)(d_nu + 2), d_nu + 4, n_tiles);
    else
      hipLaunchKernelGGL(k_pk_group_len<uint32_t>, dim3(grid_tiles), dim3(kGroupLenThreads), 0, s,
                         (const uint32_t*)o.tile_grp, (const uint32_t*)o.tfirst, (const uint32_t*)skeys, kl, n_gb,
                         glen, (unsigned long long*)rev, (unsigned long long*)(d_nu + 2), d_nu + 4, n_tiles);
    PKLAUNCH("k_pk_group_len");
    scan_add<int64_t>(glen, o.grp_off, gsums, ng + 1, s);
    PKLAUNCH("scan of group events");
    // ---- 7. fill --------------------------------------------------------
    // every event may be packed (events outside the window are not: the
    // arrays keep room for them)
    o.ev = (uint32_t*)own((size_t)N * 12, e2);
    PK(e2);
    o.desc = (uint2*)own((size_t)ng * kGroupUnits * 8, e2);
    PK(e2);
    if (in.glitch_clk > 0) {
      o.rgl = (float*)own((size_t)N * 4, e2);
      PK(e2);
    }
    {
      const bool phases = in.slot_quads > 0 && ng > 0;
      if (phases) {
        PK(hipMemcpyAsync(d_cq, in.cq_lo.data(), (size_t)n_cells * 4, hipMemcpyHostToDevice, s));
        PK(hipMemcpyAsync(d_cq + n_cells, in.cq_hi.data(), (size_t)n_cells * 4, hipMemcpyHostToDevice, s));
      }
      if (ng > 0) {
        FillArgs fa;
        fa.bins = B;
        fa.kl = kl;
        fa.skeys = skeys;
        fa.ssrc = ssrc;
        fa.gb_start = d_gbs;
        fa.gb_cell = d_gbc;
        fa.rec = rec;
        fa.rgl_g = rgl_g;
        fa.tile_grp = (const uint32_t*)o.tile_grp;
        fa.tfirst = o.tfirst;
        fa.grp_off = o.grp_off;
        fa.ev = o.ev;
        fa.rgl = o.rgl;
        fa.desc = o.desc;
        fa.gquads = phases ? gquads : nullptr;
        fa.cq_lo = d_cq;
        fa.cq_hi = d_cq + n_cells;
        fa.max_bin = (int32_t*)d_nu + 1;
        const size_t lds = (size_t)4 << B.tile_log2;
        const unsigned gridf = grid_tiles;   // a multiple of the XCD count
        PK(launch_fill(in.unit_events <= 8, key64, fa, gridf, lds, s));
        PKLAUNCH("k_pk_fill");
      }
      // ---- 8. table phases ------------------------------------------------
      if (phases) {
        o.phases = (int4*)own((size_t)ng * sizeof(int4), e2);
        PK(e2);
        o.ph_off = (int32_t*)own((size_t)(n_tiles + 1) * 4, e2);
        PK(e2);
        hipLaunchKernelGGL(k_pk_phases, dim3((unsigned)n_tiles), dim3(64), 0, s, (const int4*)gquads,
                           (const uint32_t*)o.tile_grp, (int64_t)in.slot_quads, ph_tmp, nph, (int32_t*)d_nu + 5);
        PKLAUNCH("k_pk_phases");
        hipLaunchKernelGGL(k_pk_fill_u32, dim3(1), dim3(256), 0, s, nph + n_tiles, (int64_t)1, 0u);
        PKLAUNCH("k_pk_fill_u32");
        scan_add<uint32_t>(nph, (uint32_t*)o.ph_off, psums, n_tiles + 1, s);
        PKLAUNCH("scan of phase counts");
        hipLaunchKernelGGL(k_pk_phase_copy, dim3((unsigned)n_tiles), dim3(256), 0, s, (const int4*)ph_tmp,
                           (const uint32_t*)o.tile_grp, (const uint32_t*)o.ph_off, n_tiles, o.phases);
        PKLAUNCH("k_pk_phase_copy");
        o.slot_quads = in.slot_quads;
      }
    }
    // ---- statistics back to the host (one wait) -----------------------------
    {
      uint32_t hs[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      uint64_t nev = 0;
      uint32_t nphase = 0;
      PK(hipMemcpyAsync(hs, d_nu, sizeof hs, hipMemcpyDeviceToHost, s));
      PK(hipMemcpyAsync(&nev, o.grp_off + ng, 8, hipMemcpyDeviceToHost, s));
      if (o.ph_off) PK(hipMemcpyAsync(&nphase, o.ph_off + n_tiles, 4, hipMemcpyDeviceToHost, s));
      o.h_reg_events.resize((size_t)n_reg);
      if (n_reg > 0) PK(hipMemcpyAsync(o.h_reg_events.data(), rev, (size_t)n_reg * 8, hipMemcpyDeviceToHost, s));
      PK(hipStreamSynchronize(s));
      o.alpha_span = __builtin_bit_cast(float, hs[0]);
      o.max_bin_events = hs[1];
      o.lane_steps = (int64_t)((uint64_t)hs[2] | ((uint64_t)hs[3] << 32));
      o.max_tile_groups = (int32_t)hs[4];
      o.phases_full = o.ph_off ? (int32_t)hs[5] : 0;
      o.n_events = (int64_t)nev;
      o.n_phases = nphase;
    }
  }
  o.bytes = held;
  *out = o;
  return hipSuccess;

fail:
  (void)hipStreamSynchronize(s);
  (void)hipGetLastError();
  pack_free(&o);
  return st;
#undef PK
#undef PKLAUNCH
}

}  // namespace gtp
