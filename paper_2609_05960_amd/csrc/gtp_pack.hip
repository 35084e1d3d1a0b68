// Builds the packed, tile-major event layout described in gtp_pack.h.
//
// Steps (all on the caller's stream):
//   1. gate order: gates sorted by cell (stable, host), cut into gate blocks
//      of at most 2^gate_block_log2 gates of one cell;
//   2. k_pk_units (count pass): every gate-major lane block of 16 events is
//      walked in order and split into units wherever the gate or the time
//      tile changes; units per block are counted, then scanned;
//   3. k_pk_units (emit pass): the same walk writes one record per unit
//      (first event, gate, length, carried-in pin values) and its sort key
//      (tile, gate block, 16 - length, gate within the block);
//   4. radix sort of the unit keys (hipcub, stable);
//   5. per tile its first unit; 64 units per group; group event counts,
//      scanned into group offsets;
//   6. k_pk_fill: one wavefront per group writes the unit descriptors and
//      copies the units' events into the unit-interleaved order.
// The pack runs once per event set and bin width; its time is reported apart
// from the forward.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cstdio>
#include <vector>

#include "gtp_pack.h"

namespace gtp {
namespace {

struct UnitRec {
  int64_t src;   // gate-major index of the first event
  uint32_t x;    // cell-sorted gate | (len - 1) << 28
  uint32_t y;    // pin values before the first event | before its group << 16
};

struct KeySpec {
  int32_t gb_bits;                // bits of the gate-block field
  int32_t gb_log2;                // gates per gate block (log2)
  int32_t unit_cap;               // longest unit
  const int32_t* rank;            // gate -> cell-sorted index
  const int32_t* cell_start;      // [n_cells] first sorted index of the cell
  const int32_t* gb_base;         // [n_cells] first gate block of the cell
};

struct UnitArgs {
  EvView ev;
  const uint2* plan;
  const int32_t* gate_cell;
  const uint32_t* gate_init;
  BinSpec bins;
  KeySpec ks;
  uint32_t* counts;       // count pass: units per lane block
  const uint32_t* base;   // emit pass: first unit of each lane block
  uint64_t* keys;
  uint32_t* vals;
  UnitRec* recs;
};

template <bool kEmit>
struct UnitVisitor {
  const UnitArgs* A;
  int64_t kb;
  uint32_t n = 0;          // units closed in this block
  uint32_t init = 0;
  int32_t gs = 0;          // cell-sorted gate index
  uint32_t gblock = 0;
  uint32_t gin = 0;        // index of the gate within its gate block
  bool open = false;
  int64_t u_src = 0;
  int32_t u_len = 0;
  int64_t u_tile = 0;
  uint32_t u_st = 0;

  __device__ __forceinline__ void close() {
    if (!open) return;
    if (kEmit) {
      const uint32_t u = A->base[kb] + n;
      // (tile, gate block, 16 - length, gate within the block): lanes of one
      // length class read neighbouring gate records
      const uint64_t key = ((uint64_t)u_tile << (A->ks.gb_bits + 5 + A->ks.gb_log2)) |
                           ((uint64_t)gblock << (5 + A->ks.gb_log2)) | ((uint64_t)(16 - u_len) << A->ks.gb_log2) |
                           (uint64_t)gin;
      A->keys[u] = key;
      A->vals[u] = u;
      UnitRec r;
      r.src = u_src;
      r.x = (uint32_t)gs | ((uint32_t)(u_len - 1) << 28);
      r.y = u_st;
      A->recs[u] = r;
    }
    ++n;
    open = false;
  }
  __device__ __forceinline__ void begin_gate(int64_t g, uint32_t) {
    init = A->gate_init[g];
    const int32_t c = A->gate_cell[g];
    gs = A->ks.rank[g];
    gblock = (uint32_t)(A->ks.gb_base[c] + ((gs - A->ks.cell_start[c]) >> A->ks.gb_log2));
    gin = (uint32_t)(gs - A->ks.cell_start[c]) & ((1u << A->ks.gb_log2) - 1u);
    open = false;
  }
  __device__ __forceinline__ void end_gate(int64_t) { close(); }
  __device__ __forceinline__ void event(int64_t e, int64_t t, int, int, float, uint32_t par_gs, uint32_t par) {
    const BinSpec& B = A->bins;
    if (t < 0 || t >= B.t_end) {  // outside the window: not packed
      close();
      return;
    }
    const int64_t tile = bin_of(t, B) >> B.tile_log2;
    if (open && tile == u_tile && u_len < A->ks.unit_cap) {
      ++u_len;
      return;
    }
    close();
    open = true;
    u_src = e;
    u_len = 1;
    u_tile = tile;
    u_st = ((init ^ par) & 0xffffu) | (((init ^ par_gs) & 0xffffu) << 16);
  }
};

template <bool kEmit>
__global__ void __launch_bounds__(kFwdThreads) k_pk_units(UnitArgs a, int64_t n_blocks) {
  const int64_t kb = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (kb >= n_blocks) return;
  UnitVisitor<kEmit> vis;
  vis.A = &a;
  vis.kb = kb;
  walk_block(kb, a.ev, a.plan, vis);
  if (!kEmit) a.counts[kb] = vis.n;
}

__global__ void __launch_bounds__(256) k_pk_fill_u32(uint32_t* p, int64_t n, uint32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// First sorted unit of every non-empty tile.
__global__ void __launch_bounds__(256) k_pk_tile_first(const uint64_t* skey, int64_t nu, int32_t shift,
                                                       uint32_t* tfirst) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nu) return;
  const uint64_t t = skey[j] >> shift;
  if (j == 0 || (skey[j - 1] >> shift) != t) tfirst[t] = (uint32_t)j;
}

// First sorted unit of every non-empty (tile, gate block) region.
__global__ void __launch_bounds__(256) k_pk_region_first(const uint64_t* skey, int64_t nu, int32_t gb_bits, int32_t low,
                                                         int32_t n_gb, uint32_t* rfirst) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nu) return;
  auto region = [&](uint64_t k) -> int64_t {
    return (int64_t)(k >> (gb_bits + low)) * n_gb + (int64_t)((k >> low) & ((1ull << gb_bits) - 1ull));
  };
  const int64_t r = region(skey[j]);
  if (j == 0 || region(skey[j - 1]) != r) rfirst[r] = (uint32_t)j;
}

// Event count of every sorted unit (for the per-region event counts).
__global__ void __launch_bounds__(256) k_pk_sorted_len(const uint32_t* sidx, const UnitRec* recs, int64_t nu,
                                                       uint32_t* slen) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j > nu) return;
  slen[j] = (j < nu) ? (recs[sidx[j]].x >> 28) + 1u : 0u;
}

__global__ void __launch_bounds__(256) k_pk_region_events(const uint64_t* uoff, const uint32_t* rfirst, int64_t n_reg,
                                                          int64_t* rev) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n_reg) return;
  rev[r] = (int64_t)(uoff[rfirst[r + 1]] - uoff[rfirst[r]]);
}

__device__ __forceinline__ int32_t tile_of_group(const int32_t* tile_grp, int32_t n_tiles, int64_t gi) {
  int32_t lo = 0, hi = n_tiles;  // invariant: tile_grp[lo] <= gi < tile_grp[hi]
  while (hi - lo > 1) {
    const int32_t mid = (lo + hi) >> 1;
    if ((int64_t)tile_grp[mid] <= gi) lo = mid; else hi = mid;
  }
  return lo;
}

// Events of each group (for the offsets) and its longest unit (the number of
// lane steps the group costs a wavefront).
__global__ void __launch_bounds__(256) k_pk_group_len(const int32_t* tile_grp, const uint32_t* tfirst, int32_t n_tiles,
                                                      const uint32_t* sidx, const UnitRec* recs, int64_t n_groups,
                                                      int64_t* glen, uint8_t* gmax) {
  const int64_t gi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gi > n_groups) return;
  if (gi == n_groups) {
    glen[gi] = 0;
    return;
  }
  const int32_t k = tile_of_group(tile_grp, n_tiles, gi);
  const int64_t j0 = (int64_t)tfirst[k] + (gi - tile_grp[k]) * kGroupUnits;
  const int64_t j1 = min(j0 + kGroupUnits, (int64_t)tfirst[k + 1]);
  int64_t s = 0;
  int mx = 0;
  for (int64_t j = j0; j < j1; ++j) {
    const int len = (int)(recs[sidx[j]].x >> 28) + 1;
    s += len;
    mx = max(mx, len);
  }
  glen[gi] = s;
  gmax[gi] = (uint8_t)mx;
}

struct FillArgs {
  EvView ev;
  BinSpec bins;
  LibView lib;                // device pointers of the library image
  const int32_t* gcell;
  const int32_t* tile_grp;
  const uint32_t* tfirst;
  const uint32_t* sidx;
  const UnitRec* recs;
  const int64_t* grp_off;
  int64_t n_groups;
  uint32_t* w32;
  uint32_t* row;
  float* alpha;
  uint2* desc;
  int64_t* dsrc;
  int32_t* dbg_state;         // optional, gate-major: state before the event's group
  int64_t* dbg_bin;           // optional, gate-major: bin of the event
  int32_t* alpha_span;        // max over events of |1 - alpha| + |alpha| (FP32 bits; positive floats order as ints)
};

// One wavefront per group: the unit descriptors, and every event's record in
// the unit-interleaved order. The lane of a unit tracks its gate's pin values
// from the carried-in values, as the gate-major walk does: the table is
// selected by the input state before the event's timestamp group, the
// leakage state after the event is the input state once the event's pin has
// toggled.
__global__ void __launch_bounds__(256) k_pk_fill(FillArgs a) {
  const int64_t gi = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kGroupUnits;
  const int lane = (int)(threadIdx.x & (kGroupUnits - 1));
  if (gi >= a.n_groups) return;  // whole wavefronts exit together
  const BinSpec& B = a.bins;
  const int32_t k = tile_of_group(a.tile_grp, B.n_tiles, gi);
  const int64_t j = (int64_t)a.tfirst[k] + (gi - a.tile_grp[k]) * kGroupUnits + lane;
  const bool act = j < (int64_t)a.tfirst[k + 1];
  UnitRec r{-1, 0xffffffffu, 0u};
  if (act) r = a.recs[a.sidx[j]];
  const int cell = act ? a.gcell[r.x & 0x0fffffffu] : 0;
  // descriptor: y = pin values before the unit's first event | cell << 16
  a.desc[gi * kGroupUnits + lane] = make_uint2(r.x, (r.y & 0xffffu) | ((uint32_t)cell << 16));
  a.dsrc[gi * kGroupUnits + lane] = r.src;
  const int len = act ? (int)(r.x >> 28) + 1 : 0;
  const CellMeta cm = a.lib.meta[cell];
  const uint32_t in_mask = (1u << cm.n_in) - 1u;
  const float* axis = a.lib.slew + cm.axis_off;
  const float* inv = a.lib.slew_inv + cm.axis_off;
  const int32_t qstride = a.lib.n_load - 1;
  uint32_t cur = r.y & 0xffffu;   // pin values before the unit's first event
  uint32_t gsv = r.y >> 16;       // pin values before that event's timestamp group
  int64_t tprev = 0;
  int64_t off = a.grp_off[gi];
  float span = 1.0f;   // |1 - alpha| + |alpha| of the lane's events (1 inside the axis)
  for (int kk = 0; kk < kLaneEvents; ++kk) {
    const bool on = len > kk;
    const uint64_t m = __ballot(on);
    if (m == 0) break;
    if (on) {
      const uint32_t lo = (uint32_t)m, hi = (uint32_t)(m >> 32);
      const int64_t pos = off + __builtin_amdgcn_mbcnt_hi(hi, __builtin_amdgcn_mbcnt_lo(lo, 0u));
      const int64_t e = r.src + kk;
      const int64_t t = a.ev.t[e];
      const uint32_t pb = a.ev.pb[e];
      if (kk > 0 && t != tprev) gsv = cur;
      tprev = t;
      const uint32_t pin = min(pb >> 1, (uint32_t)kMaxPin);
      const uint32_t v = pb & 1u;
      const uint32_t st = gsv & in_mask;
      cur ^= 1u << pin;
      const int64_t bin = bin_of(t, B);
      const uint32_t bl = (uint32_t)(bin - ((int64_t)k << B.tile_log2));
      const uint32_t rr = (uint32_t)(t - bin * B.D);
      int i;
      float al;
      slew_segment(axis, inv, a.lib.n_slew, a.ev.slew[e], i, al);
      const uint32_t q = (uint32_t)(a.lib.map_q[cm.map_off + 2 * (int)st + (int)v] + i * qstride);
      a.w32[pos] = (bl << B.r_bits) | rr | ((cur & in_mask) << kStateShift);
      a.row[pos] = q | ((pin == (uint32_t)cm.n_in ? 1u : 0u) << kOutBit) | (v << 31);
      a.alpha[pos] = al;
      span = fmaxf(span, fabsf(1.0f - al) + fabsf(al));
      if (a.dbg_state) {
        a.dbg_state[e] = (int32_t)st;
        a.dbg_bin[e] = bin;
      }
    }
    off += __popcll(m);
  }
  for (int o = 32; o > 0; o >>= 1) span = fmaxf(span, __shfl_xor(span, o, 64));
  if (lane == 0) atomicMax(a.alpha_span, __float_as_int(span));
}

// Largest number of events in one bin: one workgroup per tile counts the
// tile's packed events per bin in LDS (the in-tile bin is in the event
// word), then one atomic max per tile.
__global__ void __launch_bounds__(256) k_pk_bin_max(const uint32_t* w32, const int64_t* grp_off,
                                                    const int32_t* tile_grp, int32_t tile_log2, int32_t r_bits,
                                                    int32_t* out) {
  extern __shared__ int32_t hist[];
  const int nb = 1 << tile_log2;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) hist[i] = 0;
  __syncthreads();
  const int32_t k = blockIdx.x;
  const int64_t e0 = grp_off[tile_grp[k]], e1 = grp_off[tile_grp[k + 1]];
  for (int64_t e = e0 + threadIdx.x; e < e1; e += blockDim.x)
    atomicAdd(&hist[(w32[e] & kTimeMask) >> r_bits], 1);
  __syncthreads();
  int mx = 0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) mx = max(mx, hist[i]);
  for (int o = 32; o > 0; o >>= 1) mx = max(mx, __shfl_xor(mx, o, 64));
  if ((threadIdx.x & 63) == 0 && mx > 0) atomicMax(out, mx);
}

// First and last cell among a group's units (-1 for an empty group); the
// lanes of a group are in gate-block order, so cells do not decrease.
__global__ void __launch_bounds__(256) k_pk_group_cells(const uint2* desc, const int32_t* gcell, int64_t n_groups,
                                                        int2* cells) {
  const int64_t gi = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kGroupUnits;
  const int lane = (int)(threadIdx.x & (kGroupUnits - 1));
  if (gi >= n_groups) return;
  const uint2 d = desc[gi * kGroupUnits + lane];
  const bool v = d.x != 0xffffffffu;
  const uint64_t m = __ballot(v);
  if (m == 0) {
    if (lane == 0) cells[gi] = make_int2(-1, -1);
    return;
  }
  const int first = __ffsll((unsigned long long)m) - 1;
  const int last = 63 - __clzll((long long)m);
  if (lane == first) cells[gi].x = gcell[d.x & 0x0fffffffu];
  if (lane == last) cells[gi].y = gcell[d.x & 0x0fffffffu];
}

// Output nets and initial pin values in cell-sorted gate order (the per-call
// gate records then read them contiguously).
__global__ void __launch_bounds__(256) k_pk_gate_sorted(const int32_t* gperm, const int32_t* gate_out,
                                                        const uint32_t* gate_init, int64_t n_gates, int32_t* gout,
                                                        uint32_t* ginit) {
  const int64_t gs = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gs >= n_gates) return;
  const int32_t g = gperm[gs];
  gout[gs] = gate_out[g];
  ginit[gs] = gate_init[g];
}

// Sort key of gate g for the cell-sorted gate order: cell, then decreasing
// weight (its event count unless weights are given; capped at 2^20 - 1),
// then the gate index (n_cells < 2^16, gates < 2^28).
constexpr int64_t kWeightCap = (1 << 20) - 1;
__global__ void __launch_bounds__(256) k_pk_gate_keys(const int32_t* gate_cell, const int64_t* gate_off,
                                                      const int64_t* weight, int64_t n_gates, uint64_t* keys) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n_gates) return;
  const int64_t w = weight ? weight[g] : gate_off[g + 1] - gate_off[g];
  const uint64_t wq = (uint64_t)(kWeightCap - min(max(w, (int64_t)0), kWeightCap));
  keys[g] = ((uint64_t)(uint32_t)gate_cell[g] << 48) | (wq << 28) | (uint64_t)g;
}

// The sorted keys as the permutation (sorted index -> gate), its inverse and
// each sorted gate's cell.
__global__ void __launch_bounds__(256) k_pk_gate_order(const uint64_t* skeys, int64_t n_gates, int32_t* perm,
                                                       int32_t* rank, int32_t* pcell) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n_gates) return;
  const uint64_t k = skeys[r];
  const int32_t g = (int32_t)(k & ((1u << 28) - 1u));
  perm[r] = g;
  rank[g] = (int32_t)r;
  pcell[r] = (int32_t)(k >> 48);
}

int ceil_log2_u64(uint64_t x) {
  int l = 0;
  while ((1ull << l) < x) ++l;
  return l;
}

}  // namespace

void pack_free(PackOut* o) {
  void* ps[] = {o->w32,   o->row,   o->alpha, o->desc,      o->dsrc,   o->grp_off, o->tile_grp, o->gperm,
                o->gcell, o->gout, o->ginit, o->reg_first, o->tfirst, o->phases, o->ph_off};
  for (void* p : ps)
    if (p) (void)hipFree(p);
  *o = PackOut();
}

hipError_t pack_events(const PackIn& in, PackOut* out, char* err, size_t err_len) {
  std::vector<void*> temps;
  PackOut o;
  hipError_t st = hipSuccess;
  const hipStream_t s = in.stream;
  const int64_t G = in.ev.n_gates, N = in.ev.n;
  const int32_t n_cells = (int32_t)in.n_in.size();
  const BinSpec& B = in.bins;
  const int32_t n_tiles = B.n_tiles;
  int64_t held = 0;

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

  auto tmp = [&](size_t bytes, hipError_t& e) -> void* {
    void* p = nullptr;
    e = hipMalloc(&p, std::max<size_t>(bytes, 256));
    if (e == hipSuccess) temps.push_back(p);
    return p;
  };
  auto own = [&](size_t bytes, hipError_t& e) -> void* {
    void* p = nullptr;
    bytes = std::max<size_t>(bytes, 256);
    e = hipMalloc(&p, bytes);
    if (e == hipSuccess) held += (int64_t)bytes;
    return p;
  };

  {
    // ---- 1. gate order (host) -------------------------------------------
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
    const int gb_bits = ceil_log2_u64((uint64_t)n_gb);
    const int tile_bits = std::max(1, ceil_log2_u64((uint64_t)n_tiles));
    const int low = 5 + in.gate_block_log2;   // length and gate-within-block fields
    const int key_bits = tile_bits + gb_bits + low;
    if (key_bits > 64) {
      snprintf(err, err_len, "pack: sort key of %d bits", key_bits);
      return hipErrorInvalidValue;
    }
    hipError_t e2;
    int32_t* d_rank = (int32_t*)tmp((size_t)G * 4, e2);
    PK(e2);
    int32_t* d_cs = (int32_t*)tmp((size_t)n_cells * 4, e2);
    PK(e2);
    int32_t* d_gbb = (int32_t*)tmp((size_t)n_cells * 4, e2);
    PK(e2);
    o.gperm = (int32_t*)own((size_t)G * 4, e2);
    PK(e2);
    o.gcell = (int32_t*)own((size_t)G * 4, e2);
    PK(e2);
    o.gout = (int32_t*)own((size_t)G * 4, e2);
    PK(e2);
    o.ginit = (uint32_t*)own((size_t)G * 4, e2);
    PK(e2);
    if (G > 0) {
      // Gates in cell order and, within a cell, by decreasing event count (or
      // the given weights; ties by gate index): the gates active in most time
      // tiles sit together, so the gate records one wavefront gathers share
      // cache lines.
      uint64_t* gk = (uint64_t*)tmp((size_t)G * 8, e2);
      PK(e2);
      uint64_t* gks = (uint64_t*)tmp((size_t)G * 8, e2);
      PK(e2);
      int64_t* d_wt = nullptr;
      if ((int64_t)in.gate_weight.size() == G) {
        d_wt = (int64_t*)tmp((size_t)G * 8, e2);
        PK(e2);
        PK(hipMemcpyAsync(d_wt, in.gate_weight.data(), (size_t)G * 8, hipMemcpyHostToDevice, s));
      }
      const dim3 gg((unsigned)((G + 255) / 256));
      hipLaunchKernelGGL(k_pk_gate_keys, gg, dim3(256), 0, s, in.gate_cell, in.ev.gate_off, d_wt, (int64_t)G, gk);
      PKLAUNCH("k_pk_gate_keys");
      size_t tb = 0;
      PK(hipcub::DeviceRadixSort::SortKeys(nullptr, tb, gk, gks, (int)G, 0, 64, s));
      void* tsort = tmp(tb, e2);
      PK(e2);
      PK(hipcub::DeviceRadixSort::SortKeys(tsort, tb, gk, gks, (int)G, 0, 64, s));
      hipLaunchKernelGGL(k_pk_gate_order, gg, dim3(256), 0, s, gks, (int64_t)G, o.gperm, d_rank, o.gcell);
      PKLAUNCH("k_pk_gate_order");
      hipLaunchKernelGGL(k_pk_gate_sorted, dim3((unsigned)((G + 255) / 256)), dim3(256), 0, s, o.gperm, in.gate_out,
                         in.gate_init, (int64_t)G, o.gout, o.ginit);
      PKLAUNCH("k_pk_gate_sorted");
    }
    PK(hipMemcpyAsync(d_cs, cell_start.data(), (size_t)n_cells * 4, hipMemcpyHostToDevice, s));
    PK(hipMemcpyAsync(d_gbb, gb_base.data(), (size_t)n_cells * 4, hipMemcpyHostToDevice, s));

    // ---- 2-3. units -----------------------------------------------------
    const int64_t n_blocks = (N + kLaneEvents - 1) / kLaneEvents;
    UnitArgs ua;
    ua.ev = in.ev;
    ua.plan = in.plan_blk;
    ua.gate_cell = in.gate_cell;
    ua.gate_init = in.gate_init;
    ua.bins = B;
    ua.ks.gb_bits = gb_bits;
    ua.ks.gb_log2 = in.gate_block_log2;
    ua.ks.unit_cap = in.unit_events;
    ua.ks.rank = d_rank;
    ua.ks.cell_start = d_cs;
    ua.ks.gb_base = d_gbb;
    uint32_t* counts = (uint32_t*)tmp((size_t)(n_blocks + 1) * 4, e2);
    PK(e2);
    uint32_t* ubase = (uint32_t*)tmp((size_t)(n_blocks + 1) * 4, e2);
    PK(e2);
    ua.counts = counts;
    ua.base = ubase;
    ua.keys = nullptr;
    ua.vals = nullptr;
    ua.recs = nullptr;
    int64_t NU = 0;
    if (n_blocks > 0) {
      const unsigned gridb = (unsigned)((n_blocks + kFwdThreads - 1) / kFwdThreads);
      hipLaunchKernelGGL((k_pk_units<false>), dim3(gridb), dim3(kFwdThreads), 0, s, ua, n_blocks);
      PKLAUNCH("k_pk_units<count>");
      hipLaunchKernelGGL(k_pk_fill_u32, dim3(1), dim3(256), 0, s, counts + n_blocks, (int64_t)1, 0u);
      PKLAUNCH("k_pk_fill_u32");
      size_t tb = 0;
      PK(hipcub::DeviceScan::ExclusiveSum(nullptr, tb, counts, ubase, (int)(n_blocks + 1), s));
      void* tscan = tmp(tb, e2);
      PK(e2);
      PK(hipcub::DeviceScan::ExclusiveSum(tscan, tb, counts, ubase, (int)(n_blocks + 1), s));
      uint32_t tot = 0;
      PK(hipMemcpyAsync(&tot, ubase + n_blocks, 4, hipMemcpyDeviceToHost, s));
      PK(hipStreamSynchronize(s));
      NU = tot;
    }
    o.n_units = NU;
    uint64_t* keys = (uint64_t*)tmp((size_t)NU * 8, e2);
    PK(e2);
    uint64_t* skeys = (uint64_t*)tmp((size_t)NU * 8, e2);
    PK(e2);
    uint32_t* vals = (uint32_t*)tmp((size_t)NU * 4, e2);
    PK(e2);
    uint32_t* sidx = (uint32_t*)tmp((size_t)NU * 4, e2);
    PK(e2);
    UnitRec* recs = (UnitRec*)tmp((size_t)NU * sizeof(UnitRec), e2);
    PK(e2);
    if (NU > 0) {
      ua.keys = keys;
      ua.vals = vals;
      ua.recs = recs;
      const unsigned gridb = (unsigned)((n_blocks + kFwdThreads - 1) / kFwdThreads);
      hipLaunchKernelGGL((k_pk_units<true>), dim3(gridb), dim3(kFwdThreads), 0, s, ua, n_blocks);
      PKLAUNCH("k_pk_units<emit>");
      // ---- 4. sort ------------------------------------------------------
      size_t tb = 0;
      PK(hipcub::DeviceRadixSort::SortPairs(nullptr, tb, keys, skeys, vals, sidx, (int)NU, 0, key_bits, s));
      void* tsort = tmp(tb, e2);
      PK(e2);
      PK(hipcub::DeviceRadixSort::SortPairs(tsort, tb, keys, skeys, vals, sidx, (int)NU, 0, key_bits, s));
    }
    // ---- 5. tiles and groups -------------------------------------------
    uint32_t* tfirst = (uint32_t*)own((size_t)(n_tiles + 1) * 4, e2);
    PK(e2);
    o.tfirst = tfirst;
    hipLaunchKernelGGL(k_pk_fill_u32, dim3((unsigned)((n_tiles + 1 + 255) / 256)), dim3(256), 0, s, tfirst,
                       (int64_t)(n_tiles + 1), (uint32_t)NU);
    PKLAUNCH("k_pk_fill_u32");
    if (NU > 0) {
      hipLaunchKernelGGL(k_pk_tile_first, dim3((unsigned)((NU + 255) / 256)), dim3(256), 0, s, skeys, NU,
                         gb_bits + low, tfirst);
      PKLAUNCH("k_pk_tile_first");
    }
    std::vector<uint32_t> htf((size_t)n_tiles + 1);
    PK(hipMemcpyAsync(htf.data(), tfirst, (size_t)(n_tiles + 1) * 4, hipMemcpyDeviceToHost, s));
    PK(hipStreamSynchronize(s));
    for (int32_t k = n_tiles - 1; k >= 0; --k) htf[k] = std::min(htf[k], htf[k + 1]);
    std::vector<int32_t> htg((size_t)n_tiles + 1);
    int64_t ng = 0;
    int32_t maxg = 0;
    for (int32_t k = 0; k < n_tiles; ++k) {
      htg[k] = (int32_t)ng;
      const int64_t gk = ((int64_t)(htf[k + 1] - htf[k]) + kGroupUnits - 1) / kGroupUnits;
      maxg = std::max<int32_t>(maxg, (int32_t)gk);
      ng += gk;
    }
    htg[n_tiles] = (int32_t)ng;
    if (ng >= (int64_t)INT32_MAX) {
      snprintf(err, err_len, "pack: %lld groups", (long long)ng);
      st = hipErrorInvalidValue;
      goto fail;
    }
    o.n_groups = ng;
    o.max_tile_groups = maxg;
    PK(hipMemcpyAsync(tfirst, htf.data(), (size_t)(n_tiles + 1) * 4, hipMemcpyHostToDevice, s));
    o.tile_grp = (int32_t*)own((size_t)(n_tiles + 1) * 4, e2);
    PK(e2);
    PK(hipMemcpyAsync(o.tile_grp, htg.data(), (size_t)(n_tiles + 1) * 4, hipMemcpyHostToDevice, s));
    int64_t* glen = (int64_t*)tmp((size_t)(ng + 1) * 8, e2);
    PK(e2);
    o.grp_off = (int64_t*)own((size_t)(ng + 1) * 8, e2);
    PK(e2);
    uint8_t* gmax = (uint8_t*)tmp((size_t)(ng + 1), e2);
    PK(e2);
    hipLaunchKernelGGL(k_pk_group_len, dim3((unsigned)((ng + 1 + 255) / 256)), dim3(256), 0, s, o.tile_grp, tfirst,
                       n_tiles, sidx, recs, ng, glen, gmax);
    PKLAUNCH("k_pk_group_len");
    {
      std::vector<uint8_t> hm((size_t)ng);
      if (ng > 0) PK(hipMemcpyAsync(hm.data(), gmax, (size_t)ng, hipMemcpyDeviceToHost, s));
      PK(hipStreamSynchronize(s));
      int64_t steps = 0;
      for (uint8_t m : hm) steps += m;
      o.lane_steps = steps;
    }
    {
      size_t tb = 0;
      PK(hipcub::DeviceScan::ExclusiveSum(nullptr, tb, glen, o.grp_off, (int)(ng + 1), s));
      void* tscan = tmp(tb, e2);
      PK(e2);
      PK(hipcub::DeviceScan::ExclusiveSum(tscan, tb, glen, o.grp_off, (int)(ng + 1), s));
    }
    int64_t nev = 0;
    PK(hipMemcpyAsync(&nev, o.grp_off + ng, 8, hipMemcpyDeviceToHost, s));
    PK(hipStreamSynchronize(s));
    o.n_events = nev;
    // ---- 5b. gate-block regions -------------------------------------------
    {
      const int64_t n_reg = (int64_t)n_tiles * n_gb;
      o.reg_first = (uint32_t*)own((size_t)(n_reg + 1) * 4, e2);
      PK(e2);
      hipLaunchKernelGGL(k_pk_fill_u32, dim3((unsigned)((n_reg + 1 + 255) / 256)), dim3(256), 0, s, o.reg_first,
                         n_reg + 1, (uint32_t)NU);
      PKLAUNCH("k_pk_fill_u32");
      if (NU > 0) {
        hipLaunchKernelGGL(k_pk_region_first, dim3((unsigned)((NU + 255) / 256)), dim3(256), 0, s, skeys, NU, gb_bits,
                           low, n_gb, o.reg_first);
        PKLAUNCH("k_pk_region_first");
      }
      std::vector<uint32_t> hrf((size_t)n_reg + 1);
      PK(hipMemcpyAsync(hrf.data(), o.reg_first, (size_t)(n_reg + 1) * 4, hipMemcpyDeviceToHost, s));
      PK(hipStreamSynchronize(s));
      for (int64_t r = n_reg - 1; r >= 0; --r) hrf[r] = std::min(hrf[r], hrf[r + 1]);
      PK(hipMemcpyAsync(o.reg_first, hrf.data(), (size_t)(n_reg + 1) * 4, hipMemcpyHostToDevice, s));
      uint32_t* slen = (uint32_t*)tmp((size_t)(NU + 1) * 4, e2);
      PK(e2);
      uint64_t* uoff = (uint64_t*)tmp((size_t)(NU + 1) * 8, e2);
      PK(e2);
      int64_t* rev = (int64_t*)tmp((size_t)std::max<int64_t>(n_reg, 1) * 8, e2);
      PK(e2);
      hipLaunchKernelGGL(k_pk_sorted_len, dim3((unsigned)((NU + 1 + 255) / 256)), dim3(256), 0, s, sidx, recs, NU, slen);
      PKLAUNCH("k_pk_sorted_len");
      size_t tb = 0;
      PK(hipcub::DeviceScan::ExclusiveSum(nullptr, tb, slen, uoff, (int)(NU + 1), s));
      void* tscan = tmp(tb, e2);
      PK(e2);
      PK(hipcub::DeviceScan::ExclusiveSum(tscan, tb, slen, uoff, (int)(NU + 1), s));
      if (n_reg > 0) {
        hipLaunchKernelGGL(k_pk_region_events, dim3((unsigned)((n_reg + 255) / 256)), dim3(256), 0, s, uoff, o.reg_first,
                           n_reg, rev);
        PKLAUNCH("k_pk_region_events");
      }
      o.h_reg_events.resize((size_t)n_reg);
      if (n_reg > 0)
        PK(hipMemcpyAsync(o.h_reg_events.data(), rev, (size_t)n_reg * 8, hipMemcpyDeviceToHost, s));
      PK(hipStreamSynchronize(s));
    }
    // ---- 6. fill --------------------------------------------------------
    int32_t* d_bounds = (int32_t*)tmp(2 * sizeof(int32_t), e2);   // [alpha span bits, max events per bin]
    PK(e2);
    {
      const int32_t init[2] = {__builtin_bit_cast(int32_t, 1.0f), 0};
      PK(hipMemcpyAsync(d_bounds, init, sizeof init, hipMemcpyHostToDevice, s));
    }
    o.w32 = (uint32_t*)own((size_t)nev * 4, e2);
    PK(e2);
    o.row = (uint32_t*)own((size_t)nev * 4, e2);
    PK(e2);
    o.alpha = (float*)own((size_t)nev * 4, e2);
    PK(e2);
    o.desc = (uint2*)own((size_t)ng * kGroupUnits * 8, e2);
    PK(e2);
    o.dsrc = (int64_t*)own((size_t)ng * kGroupUnits * 8, e2);
    PK(e2);
    if (ng > 0) {
      FillArgs fa;
      fa.ev = in.ev;
      fa.bins = B;
      fa.lib = in.lib;
      fa.gcell = o.gcell;
      fa.tile_grp = o.tile_grp;
      fa.tfirst = tfirst;
      fa.sidx = sidx;
      fa.recs = recs;
      fa.grp_off = o.grp_off;
      fa.n_groups = ng;
      fa.w32 = o.w32;
      fa.row = o.row;
      fa.alpha = o.alpha;
      fa.dbg_state = in.dbg_state;
      fa.dbg_bin = in.dbg_bin;
      fa.desc = o.desc;
      fa.dsrc = o.dsrc;
      fa.alpha_span = d_bounds;
      const int64_t threads = ng * kGroupUnits;
      hipLaunchKernelGGL(k_pk_fill, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, fa);
      PKLAUNCH("k_pk_fill");
      hipLaunchKernelGGL(k_pk_bin_max, dim3((unsigned)n_tiles), dim3(256), (size_t)4 << B.tile_log2, s, o.w32,
                         o.grp_off, o.tile_grp, B.tile_log2, B.r_bits, d_bounds + 1);
      PKLAUNCH("k_pk_bin_max");
    }
    {
      int32_t hb[2] = {0, 0};
      PK(hipMemcpyAsync(hb, d_bounds, sizeof hb, hipMemcpyDeviceToHost, s));
      PK(hipStreamSynchronize(s));
      o.alpha_span = __builtin_bit_cast(float, hb[0]);
      o.max_bin_events = hb[1];
    }
    // ---- 7. table phases ------------------------------------------------
    if (in.slot_quads > 0 && ng > 0) {
      int2* gc = (int2*)tmp((size_t)ng * 8, e2);
      PK(e2);
      const int64_t threads = ng * kGroupUnits;
      hipLaunchKernelGGL(k_pk_group_cells, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, o.desc, o.gcell,
                         ng, gc);
      PKLAUNCH("k_pk_group_cells");
      std::vector<int2> hgc((size_t)ng);
      std::vector<int32_t> htg((size_t)n_tiles + 1);
      PK(hipMemcpyAsync(hgc.data(), gc, (size_t)ng * 8, hipMemcpyDeviceToHost, s));
      PK(hipMemcpyAsync(htg.data(), o.tile_grp, (size_t)(n_tiles + 1) * 4, hipMemcpyDeviceToHost, s));
      PK(hipStreamSynchronize(s));
      const int64_t cap = in.slot_quads;
      std::vector<int4> ph;
      std::vector<int32_t> poff((size_t)n_tiles + 1, 0);
      bool all_full = true;
      for (int32_t k = 0; k < n_tiles; ++k) {
        poff[k] = (int32_t)ph.size();
        int64_t g = htg[k];
        const int64_t g1 = htg[k + 1];
        while (g < g1) {
          // a phase starts at group g and grows while the union of its
          // groups' cell table ranges fits the slot
          int64_t lo = INT64_MAX, hi = INT64_MIN;
          int64_t e = g;
          for (; e < g1; ++e) {
            const int2 cc = hgc[(size_t)e];
            if (cc.x < 0) continue;
            const int64_t l = std::min(in.cq_lo[cc.x], in.cq_lo[cc.y]), h = std::max(in.cq_hi[cc.x], in.cq_hi[cc.y]);
            const int64_t nl = std::min(lo, l), nh = std::max(hi, h);
            if (e > g && nh - nl > cap) break;
            lo = nl;
            hi = nh;
          }
          if (lo == INT64_MAX) {  // only empty groups: nothing to stage
            lo = 0;
            hi = 0;
          }
          // a single group whose cells exceed the slot keeps its first cell's
          // tables (the other lanes read the tables from global memory)
          int32_t full = 1;
          if (hi - lo > cap) {
            const int2 cc = hgc[(size_t)g];
            lo = in.cq_lo[cc.x];
            hi = std::min<int64_t>(in.cq_hi[cc.x], lo + cap);
            full = 0;
            all_full = false;
          }
          ph.push_back(make_int4((int32_t)(e - htg[k]), (int32_t)lo, (int32_t)(hi - lo), full));
          g = e;
        }
      }
      poff[n_tiles] = (int32_t)ph.size();
      o.n_phases = (int64_t)ph.size();
      o.phases_full = all_full ? 1 : 0;
      o.slot_quads = in.slot_quads;
      o.phases = (int4*)own(std::max<size_t>(ph.size(), 1) * sizeof(int4), e2);
      PK(e2);
      o.ph_off = (int32_t*)own((size_t)(n_tiles + 1) * 4, e2);
      PK(e2);
      if (!ph.empty()) PK(hipMemcpyAsync(o.phases, ph.data(), ph.size() * sizeof(int4), hipMemcpyHostToDevice, s));
      PK(hipMemcpyAsync(o.ph_off, poff.data(), poff.size() * 4, hipMemcpyHostToDevice, s));
      PK(hipStreamSynchronize(s));
    }
  }
  for (void* p : temps) (void)hipFree(p);
  o.bytes = held;
  *out = o;
  return hipSuccess;

fail:
  (void)hipStreamSynchronize(s);
  (void)hipGetLastError();
  for (void* p : temps) (void)hipFree(p);
  pack_free(&o);
  return st;
#undef PK
#undef PKLAUNCH
}

}  // namespace gtp
