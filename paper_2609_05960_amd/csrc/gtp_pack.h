// Packed event layout (built once per event set and bin width, read by every
// forward call).
//
// The waveform accumulates every event into the bin of its timestamp, so the
// forward works one time tile (2^tile_log2 consecutive bins) at a time, with
// the tile's bins privatised in LDS. The caller's events are gate-major; the
// pack regroups them by tile without losing the per-gate order the state
// tracking needs:
//
//   unit   at most 16 consecutive events (gate-major order) of one gate that
//          fall in one tile and in one 16-event block of the gate-major
//          array. Dense gates thus become many full 16-event units (the
//          "dense gates cut into time segments" of the density split);
//          sparse gates become short units. A unit carries its gate and the
//          gate's pin values before its first event and before that event's
//          timestamp group (carried-in state).
//   order  units sorted by (tile, gate block, decreasing length, gate); a
//          gate block is a run of at most 2^13 (tunable) cell-sorted gates of one cell,
//          so the units of one wavefront share a cell (table gathers stay in
//          cache), have similar lengths (lanes stay busy) and, within a
//          length, increasing gates (the per-unit gate-record loads of a
//          wavefront touch fewer cache lines).
//   group  64 consecutive units of one tile, one per lane of a wavefront. The
//          group's events are stored unit-interleaved: event k of every unit
//          longer than k, in lane order, then event k+1, ... So the k-th
//          loads of a wavefront are adjacent records.
//
// Arrays (device, owned by the ctx):
//   ev[3n]    per event, in the groups' order (group g from grp_off[g]),
//             three words: the event word (see gtp_device.h: in-tile time,
//             input state after the event), the table row (row at the slew
//             segment, output flag, value) and the slew weight (FP32 bits)
//   rgl[n]    energy factor (glitch detection on only): the glitch scaling
//             ratio of a glitch event, 1 for a regular event
//   desc[64 * n_groups]   unit descriptor: x = cell-sorted gate index
//             (bits 0..27) | (length-1) << 28, y = pin values before the
//             unit's first event (bits 0..15) | the gate's cell << 16;
//             x = 0xffffffff for an empty lane
//   grp_off[n_groups + 1] first event of each group
//   tile_grp[n_tiles + 1] first group of each tile
//   gperm[G]  cell-sorted index -> gate;  gcell[G] cell of each sorted index;
//   gout[G], ginit[G]  output net and initial pin values in sorted order
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "gtp_device.h"

namespace gtp {

constexpr int kGateBlockLog2 = 13;   // default gate-block size (log2): the adjoint holds 16 B per gate of a block in LDS

// Device memory the pack takes its temporaries from (grown on demand, kept
// by the caller between packs, freed by the caller).
struct Workspace {
  void* p = nullptr;
  size_t bytes = 0;
};

struct PackIn {
  EvView ev;                  // gate-major events (device)
  const uint2* plan_blk;      // gate-major lane-block plan (device)
  const int32_t* gate_cell;   // [G] (device)
  const int32_t* gate_out;    // [G] (device)
  const uint32_t* gate_init;  // [G] (device)
  std::vector<int32_t> h_gate_cell;  // [G] host copy
  std::vector<int32_t> n_in;         // [n_cells] inputs per cell
  LibView lib;                // library image (device pointers)
  int32_t unit_events = kLaneEvents;          // longest unit, 1..16
  int32_t gate_block_log2 = kGateBlockLog2;   // gates per gate block (log2)
  BinSpec bins;               // tile_log2 and n_tiles set
  hipStream_t stream;
  int32_t* dbg_state = nullptr;   // optional [n_events] gate-major: state before the event's group
  int64_t* dbg_bin = nullptr;     // optional [n_events] gate-major: bin of the event
  std::vector<int32_t> cq_lo, cq_hi;  // [n_cells] quad index range of each cell's tables
  // optional [G] gate weights: a cell's gates are ordered by decreasing
  // weight (empty: by this trace's event counts). Traces that share gate
  // records must share the order, so a batch passes one set of weights.
  std::vector<int64_t> gate_weight;
  int32_t slot_quads = 0;         // quads one LDS table slot holds (0: no phases)
  Workspace* ws = nullptr;        // [2] temporaries (caller-owned)
  int64_t glitch_clk = 0;         // > 0: per-event glitch factors for this clock period
  Workspace* arena = nullptr;     // optional: output arrays carved from it while it has room
  bool time_order = false;        // units of one (tile, gate block, length) ordered by the time of their
                                  // first event instead of by gate (gate blocks of at most 2^16 gates)
};

struct PackOut {
  uint32_t* ev = nullptr;     // 3 words per event (see above)
  float* rgl = nullptr;       // energy factor per event (glitch detection on), else null
  uint2* desc = nullptr;
  int64_t* grp_off = nullptr;
  int32_t* tile_grp = nullptr;
  int32_t* gperm = nullptr;
  int32_t* gcell = nullptr;
  int32_t* gout = nullptr;     // [G] output net of each cell-sorted gate
  uint32_t* ginit = nullptr;   // [G] initial pin values of each cell-sorted gate
  int64_t n_events = 0;       // events packed (valid times)
  int64_t n_units = 0;
  int64_t n_groups = 0;
  int64_t bytes = 0;          // device bytes held by the arrays above
  int32_t max_tile_groups = 0;
  int64_t lane_steps = 0;     // sum over groups of the longest unit
  // gate-block view (the adjoint's work decomposition): sorted units of
  // region r = tile * n_gb + gate block are [reg_first[r], reg_first[r+1])
  // (indices over all sorted units; tile k's units start at tfirst[k], its
  // j-th unit is lane j % 64 of group tile_grp[k] + j / 64)
  uint32_t* reg_first = nullptr;   // [n_tiles * n_gb + 1] (device)
  uint32_t* tfirst = nullptr;      // [n_tiles + 1] (device)
  int32_t n_gb = 0;
  int32_t gb_log2 = 0;
  std::vector<int32_t> h_gb_start;     // [n_gb + 1] first sorted gate of each gate block
  std::vector<int32_t> h_gb_cell;      // [n_gb] cell of each gate block
  std::vector<int64_t> h_reg_events;   // [n_tiles * n_gb] events per region
  // table phases of the forward: tile k's groups split into runs whose
  // cells' table quads [lo, lo + n) fit one LDS slot; phase p of tile k is
  // phases[ph_off[k] + p] = (end group, lo, n, full), runs cover the tile's
  // groups; full = 1 when [lo, lo + n) holds every quad the phase's groups
  // read (0 only for a group whose cells alone exceed the slot)
  int4* phases = nullptr;
  int32_t* ph_off = nullptr;       // [n_tiles + 1]
  int64_t n_phases = 0;
  int32_t phases_full = 0;         // 1: every phase is full
  int32_t slot_quads = 0;          // slot capacity the phases were cut for
  // bounds for the fixed-point range (independent of the tuning): the most
  // events in one bin and the largest |1 - alpha| + |alpha| of a slew weight
  int64_t max_bin_events = 0;
  float alpha_span = 1.0f;
  int32_t mfix = 0;                // fixed-point exponent chosen for this layout (set by the ctx)
  char* arena_lo = nullptr;        // the arena the output arrays were carved from (not freed by pack_free)
  size_t arena_len = 0;
  size_t need_bytes = 0;           // bytes of all output arrays (an arena of this size holds them all)
};

// Builds the packed layout on in.stream (synchronises it). Returns
// hipSuccess or the first HIP error; on error nothing stays allocated.
hipError_t pack_events(const PackIn& in, PackOut* out, char* err, size_t err_len);
void pack_free(PackOut* out);

}  // namespace gtp
