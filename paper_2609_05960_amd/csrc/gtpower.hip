// Host side of the C ABI declared in include/gtpower.h.
//
// Call flow of one forward (all on the ctx stream, asynchronous):
//   algo 0 (packed, tile-major):
//     k_gate_params  per gate: load-axis segment and weight, switching
//                    energy, leakage scale (cell-sorted order); sum of the
//                    initial leakage rates
//     k_fwd_packed   per time tile: every unit of the tile (see gtp_pack.h)
//                    walked by one lane, energies and leakage steps
//                    accumulated into the tile's LDS bins, bins stored
//   algo 1 (baseline):
//     k_gate_prep    per gate (gate-major order)
//     k_gate_serial  one gate per thread, global int64 atomics per event
//   scan of S, k_finalize -> FP32 power per bin
// The gate-major lane-block plan (first gate and carried parity of every 16
// events) is built in gtp_load_events; the packed layout, which depends on the
// events and the bin width, is built on the first forward after
// gtp_load_events / gtp_set_params / gtp_set_tuning and reused afterwards.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <fstream>
#include <mutex>
#include <sstream>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/gtpower.h"
#include "gtp_kernels.h"
#include "gtp_pack.h"

using namespace gtp;

// Scratch memory of gtp_forward_noalloc (the per-call buffers of one packed
// forward, carved from this array). Each GPU the library runs on holds its own
// copy until the process ends. In host code `scratch` names a host-side
// stand-in: its device address on a GPU comes from hipGetSymbolAddress, taken
// once per device at context creation (scratch_address below).
constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on hip_device (the current device); resolved on
// the first call for that device.
hipError_t scratch_address(int hip_device, void** out) {
  if (hip_device < 0 || hip_device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[hip_device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[hip_device] = p;
  }
  *out = g_scratch_ptr[hip_device];
  return hipSuccess;
}

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

}  // namespace

struct gtp_ctx_s {
  int dev = 0;
  int n_cu = 256;
  void* scratch_dev = nullptr;  // device address of `scratch` on this ctx's device
  size_t dev_total = 0;       // device memory (bytes); no single buffer can exceed it
  hipStream_t stream = nullptr;
  std::string err;
  int64_t bad_event = -1;
  std::vector<DevBuf*> bufs;
  int64_t dev_bytes = 0;

  // library
  bool lib_ok = false;
  int32_t n_cells = 0, n_slew = 0, n_load = 0, n_map = 0, n_leak = 0;
  int32_t all_pins = 0;       // the library's states cover every pin (bit I = output)
  int64_t n_tables = 0;
  int32_t lds_words = 0;
  // fixed-point range inputs (see choose_mfix): largest |table entry|, the
  // largest leakage value, the load limit and the largest |1-beta|+|beta| a
  // load within [0, load_cap] gives on any cell's load axis
  double lib_tmax = 0.0, lib_leak_max = 0.0, load_cap = 0.0, beta_span = 1.0;
  std::vector<double> h_leak_max;    // [n_cells] largest leakage value of the cell
  std::vector<int32_t> h_nin;
  std::vector<int32_t> h_cq_lo, h_cq_hi;   // per cell: quad index range of its tables
  std::vector<int32_t> h_gate_cell;  // host copy of the netlist's cells
  Workspace pk_arena{nullptr, 0};    // output arrays of the single-trace layout
  size_t pk_arena_want = 0;          // the largest layout's bytes so far
  DevBuf lib_img;             // meta | leak | map_q | slew | slew_inv
  DevBuf load_axis, load_inv, quads;
  DevBuf wide_cell, wide_pat, wide_sipl;   // cells with more than 8 state pins
  bool has_wide = false;

  // netlist
  bool net_ok = false;
  int64_t n_gates = 0, n_nets = 0;
  bool unique_out = true;   // no net has two driving gates
  double r_bound = 0.0;     // bound on the total leakage rate (fJ/ps) for scales up to GTP_MAX_LEAK_SCALE
  DevBuf gate_cell, gate_out, gate_init;

  // events
  bool ev_ok = false;
  gtp_events ev{};
  int64_t n_blocks = 0;
  DevBuf plan_blk, blk_tmp, blk_tmp2, scan_sums;

  // params
  bool par_ok = false;
  gtp_params par{};
  BinSpec bins{};

  // batched traces
  struct BatchTrace {
    gtp_events ev{};
    int64_t n_blocks = 0;
    DevBuf plan;
    BinSpec bins{};
    PackOut pk;
    double pack_ms = 0.0;
    int64_t bin_off = 0;
  };
  std::vector<BatchTrace> batch;
  bool batch_packed = false;
  int64_t batch_total_bins = 0;
  int64_t batch_items = 0;
  DevBuf b_tab, b_items, b_fin, b_X, b_S, b_tile_tot, b_tile_base;
  int64_t batch_total_tiles = 0, batch_fin_blocks = 0;
  DevBuf tun_in, tun_out;  // autotuner inputs and output
  hipStream_t cap_stream = nullptr;

  // streamed windows (gtp_stream_*): two staging slots filled on copy_stream
  struct StreamSlot {
    DevBuf gate_off, t, pb, slew;
    int64_t n = 0, t0 = 0, t1 = 0;
    hipEvent_t copied = nullptr, done = nullptr;
    bool used = false;   // done has been recorded
  };
  StreamSlot st_slot[2];
  hipStream_t copy_stream = nullptr;
  bool st_on = false, st_inside = false;
  int32_t st_validate = 0;
  int64_t st_end = 0, st_next_push = 0, st_next_step = 0;
  int st_head = 0, st_pending = 0;
  DevBuf st_init;   // the netlist's initial pin values while a stream carries its own
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  const void* gkey[3] = {nullptr, nullptr, nullptr};

  // tuning + packed layout
  gtp_tuning tun{0, 0, 0, 0, 0};
  bool pack_ok = false;
  PackOut pk;
  double pack_ms = 0.0;
  Workspace pk_ws[2];   // the pack's temporaries, kept between packs
  // the adjoint's own layout (units ordered by time within a run), built on
  // the first packed adjoint after the layout was (re)built
  bool pack_adj_ok = false;
  PackOut pk_adj;

  // kernel timing (gtp_profile_enable)
  bool prof_on = false;
  std::vector<std::string> prof_names;
  struct ProfRec { int id; hipEvent_t a, b; };
  std::vector<ProfRec> prof_recs;
  std::vector<hipEvent_t> prof_pool;
  int prof_open = -1;
  hipEvent_t prof_a = nullptr;

  // per-call work buffers
  DevBuf gprep, gparam, X, S, exS, L0, flag, first_bad;
  DevBuf l0_part, tile_tot, tile_base;   // packed forward: leakage-rate partials and tile sums
  DevBuf adj_w, adj_c, adj_exc, adj_wg, adj_gtile, adj_total, gC, gL;
  DevBuf rep_small;                       // report: totals, latest event time, peak

  // packed adjoint work items (built from the pack's region tables)
  bool adj_ok = false;
  bool adj_tab_only = false;   // every adjoint item's LDS table holds all of its cell's quads
  int64_t adj_n_items = 0;
  int32_t adj_max_gb = 0;   // gates in the largest gate block
  DevBuf adj_items, adj_entries, adj_gbs, adj_gbrow, adj_gbrows, adj_part;
};

namespace {

gtp_status fail(gtp_ctx c, gtp_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  return s;
}

#define HIPCHK(ctx, call)                                                                          \
  do {                                                                                             \
    hipError_t e_ = (call);                                                                        \
    if (e_ != hipSuccess) return fail((ctx), GTP_ERR_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

#define LAUNCHCHK(ctx, name)                                                                                     \
  do {                                                                                                           \
    hipError_t e_ = hipGetLastError();                                                                           \
    if (e_ != hipSuccess) return fail((ctx), GTP_ERR_HIP, "launch of %s failed: %s", name, hipGetErrorString(e_)); \
  } while (0)

#define TRY(...)                     \
  do {                               \
    gtp_status s_ = (__VA_ARGS__);   \
    if (s_ != GTP_OK) return s_;     \
  } while (0)

hipEvent_t prof_event(gtp_ctx c) {
  if (!c->prof_pool.empty()) {
    hipEvent_t e = c->prof_pool.back();
    c->prof_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return e;
}

void prof_begin(gtp_ctx c, const char* name) {
  if (!c->prof_on) return;
  int id = -1;
  for (size_t i = 0; i < c->prof_names.size(); ++i)
    if (c->prof_names[i] == name) id = (int)i;
  if (id < 0) {
    id = (int)c->prof_names.size();
    c->prof_names.push_back(name);
  }
  c->prof_open = id;
  c->prof_a = prof_event(c);
  if (c->prof_a) (void)hipEventRecord(c->prof_a, c->stream);
}

void prof_end(gtp_ctx c) {
  if (!c->prof_on || c->prof_open < 0) return;
  hipEvent_t b = prof_event(c);
  if (b && c->prof_a) {
    (void)hipEventRecord(b, c->stream);
    c->prof_recs.push_back({c->prof_open, c->prof_a, b});
  }
  c->prof_open = -1;
  c->prof_a = nullptr;
}

void prof_clear(gtp_ctx c) {
  for (auto& r : c->prof_recs) {
    c->prof_pool.push_back(r.a);
    c->prof_pool.push_back(r.b);
  }
  c->prof_recs.clear();
}

// Launch on the ctx stream; with profiling on, bracketed by HIP events.
#define LAUNCH(c, name, kern, grid, block, lds, ...)                      \
  do {                                                                    \
    prof_begin((c), name);                                                \
    hipLaunchKernelGGL(kern, grid, block, lds, (c)->stream, __VA_ARGS__); \
    LAUNCHCHK((c), name);                                                 \
    prof_end((c));                                                        \
  } while (0)

void drop_graph(gtp_ctx c);

gtp_status ensure(gtp_ctx c, DevBuf& b, size_t bytes) {
  if (bytes == 0) bytes = 256;
  if (b.bytes >= bytes) return GTP_OK;
  if (c->dev_total > 0 && bytes > c->dev_total)
    return fail(c, GTP_ERR_OUT_OF_MEMORY, "a buffer of %zu bytes exceeds the device memory (%zu bytes)", bytes,
                c->dev_total);
  if (b.p) {
    // a recorded graph may hold this buffer's address: it is recorded again
    // on its next use
    drop_graph(c);
    (void)hipStreamSynchronize(c->stream);
    (void)hipFree(b.p);
    c->dev_bytes -= (int64_t)b.bytes;
    b.p = nullptr;
    b.bytes = 0;
  }
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess || !p) {
    (void)hipGetLastError();
    return fail(c, GTP_ERR_OUT_OF_MEMORY, "device allocation of %zu bytes failed", bytes);
  }
  b.p = p;
  b.bytes = bytes;
  c->dev_bytes += (int64_t)bytes;
  return GTP_OK;
}

void release(gtp_ctx c, DevBuf& b) {
  if (b.p) {
    (void)hipFree(b.p);
    c->dev_bytes -= (int64_t)b.bytes;
  }
  b.p = nullptr;
  b.bytes = 0;
}

template <class T>
T* ptr(DevBuf& b) {
  return reinterpret_cast<T*>(b.p);
}

inline unsigned grid_for(int64_t n, int threads) { return (unsigned)((n + threads - 1) / threads); }

gtp_status fill_u64(gtp_ctx c, void* p, int64_t n, unsigned long long v) {
  if (n <= 0) return GTP_OK;
  LAUNCH(c, "k_fill_u64", k_fill_u64, dim3(grid_for(n, 256)), dim3(256), 0, (unsigned long long*)p, n, v);
  return GTP_OK;
}

// exclusive scan of n items of T (in -> out), three passes
template <class T, class Op>
gtp_status scan_exclusive(gtp_ctx c, const T* in, T* out, int64_t n, T ident, Op op) {
  if (n <= 0) return GTP_OK;
  const int64_t nt = (n + kScanTile - 1) / kScanTile;
  TRY(ensure(c, c->scan_sums, (size_t)nt * sizeof(T)));
  T* sums = ptr<T>(c->scan_sums);
  LAUNCH(c, "k_scan_tiles", (k_scan_tiles<T, Op>), dim3((unsigned)nt), dim3(kScanThreads), 0, in, out, sums, n, ident, op);
  if (nt > 1) {
    LAUNCH(c, "k_scan_sums", (k_scan_sums<T, Op>), dim3(1), dim3(kScanThreads), 0, sums, nt, ident, op);
    LAUNCH(c, "k_scan_add", (k_scan_add<T, Op>), dim3(grid_for(n, 256)), dim3(256), 0, out, (const T*)sums, n, op);
  }
  return GTP_OK;
}

LibView lib_view(gtp_ctx c) {
  LibView L;
  const uint32_t* img = ptr<uint32_t>(c->lib_img);
  L.meta = reinterpret_cast<const CellMeta*>(img);
  const int32_t nl = c->n_cells * c->n_load;
  L.leak = reinterpret_cast<const float*>(img + 4 * c->n_cells);
  L.load = L.leak + c->n_leak;
  L.load_inv = L.load + nl;
  L.map_q = reinterpret_cast<const int32_t*>(L.load_inv + nl);
  L.slew = reinterpret_cast<const float*>(L.map_q + c->n_map);
  L.slew_inv = L.slew + c->n_cells * c->n_slew;
  L.quads = ptr<float4>(c->quads);
  L.n_cells = c->n_cells;
  L.n_slew = c->n_slew;
  L.n_load = c->n_load;
  L.n_map = c->n_map;
  L.n_leak = c->n_leak;
  L.lds_words = c->lds_words;
  L.lds_words_ml = 4 * c->n_cells + c->n_leak + 2 * nl;
  L.all_pins = c->all_pins;
  L.wide.cell = c->has_wide ? ptr<WideCell>(c->wide_cell) : nullptr;
  L.wide.pat = c->has_wide ? ptr<uint2>(c->wide_pat) : nullptr;
  L.wide.sipl = c->has_wide ? ptr<uint8_t>(c->wide_sipl) : nullptr;
  return L;
}

float rate_scale_of(int32_t m) { return (float)(std::ldexp(1.0, m) * 1e-6); }

// Exponent for kernels whose fixed-point values are not used (the adjoint
// and per-event trace of the gate-major path read only the gate state and the
// interpolation weights).
constexpr int32_t kAnyMfix = 32;
constexpr int32_t kMaxMfix = 40;   // energy unit 2^-40 fJ at most
constexpr int32_t kMinMfix = 30;   // below this the quantised leakage rates lose the 1e-5 budget
constexpr int32_t kSiplMaxPins = 16;   // direct per-state arrays up to this many state pins (Sec. 4.1)

LutArgs lut_args(gtp_ctx c, int32_t m) {
  LutArgs A;
  A.quads = ptr<float4>(c->quads);
  A.n_slew = c->n_slew;
  A.n_load = c->n_load;
  A.rate_scale = rate_scale_of(m);
  A.two_sh = (float)std::ldexp(1.0, m - 32);
  return A;
}

EvView ev_view(gtp_ctx c) {
  EvView E;
  E.t = c->ev.t_ps;
  E.pb = c->ev.pin_bit;
  E.slew = c->ev.slew_ps;
  E.gate_off = c->ev.gate_off;
  E.n = c->ev.n_events;
  E.n_gates = c->n_gates;
  return E;
}

int ceil_log2(uint64_t x) {
  int l = 0;
  while ((1ull << l) < x) ++l;
  return l;
}

Div32 make_div32(uint32_t d) {
  Div32 r;
  const int l = ceil_log2(d);
  const uint64_t m = ((((uint64_t)1 << l) - d) << 32) / d + 1;
  r.m = (uint32_t)m;
  r.s1 = std::min(l, 1);
  r.s2 = std::max(l - 1, 0);
  return r;
}

gtp_status need(gtp_ctx c, bool lib, bool net, bool ev, bool par) {
  if (!c) return GTP_ERR_INVALID_ARG;
  if (c->st_on && !c->st_inside)
    return fail(c, GTP_ERR_INVALID_ARG, "a stream is open: only gtp_stream_push/step/end until gtp_stream_end");
  if (lib && !c->lib_ok) return fail(c, GTP_ERR_NOT_LOADED, "no library loaded");
  if (net && !c->net_ok) return fail(c, GTP_ERR_NOT_LOADED, "no netlist loaded");
  if (ev && !c->ev_ok) return fail(c, GTP_ERR_NOT_LOADED, "no events loaded");
  if (par && !c->par_ok) return fail(c, GTP_ERR_NOT_LOADED, "no parameters set");
  return GTP_OK;
}

// ----------------------------------------------------------------------------
// plan
// ----------------------------------------------------------------------------
// Gate-major lane-block plan of an event set: first gate of every 16 events
// and the toggle parity that gate carries into the block.
gtp_status block_plan_for(gtp_ctx c, const gtp_events& ev, DevBuf& plan_buf, int64_t& n_blocks) {
  const int64_t N = ev.n_events;
  n_blocks = (N + kLaneEvents - 1) / kLaneEvents;
  if (n_blocks == 0) return GTP_OK;
  TRY(ensure(c, plan_buf, (size_t)n_blocks * sizeof(uint2)));
  TRY(ensure(c, c->blk_tmp, (size_t)n_blocks * sizeof(uint32_t)));
  TRY(ensure(c, c->blk_tmp2, (size_t)n_blocks * sizeof(uint32_t)));
  uint2* plan = ptr<uint2>(plan_buf);
  LAUNCH(c, "k_plan_block_gate", k_plan_block_gate, dim3(grid_for(n_blocks, 256)), dim3(256), 0, ev.gate_off, c->n_gates, N, plan, n_blocks);
  LAUNCH(c, "k_plan_block_xor", k_plan_block_xor, dim3(grid_for(n_blocks, 256)), dim3(256), 0, ev.pin_bit, N, ptr<uint32_t>(c->blk_tmp), n_blocks);
  TRY(scan_exclusive<uint32_t, OpXor>(c, ptr<uint32_t>(c->blk_tmp), ptr<uint32_t>(c->blk_tmp2), n_blocks, 0u,
                                      OpXor()));
  LAUNCH(c, "k_plan_block_carry", k_plan_block_carry, dim3(grid_for(n_blocks, 256)), dim3(256), 0, ev.gate_off, ev.pin_bit, (const uint32_t*)ptr<uint32_t>(c->blk_tmp2), plan, n_blocks);
  return GTP_OK;
}

gtp_status build_block_plan(gtp_ctx c) { return block_plan_for(c, c->ev, c->plan_blk, c->n_blocks); }

// Bins per tile: the largest power of two (at most 2^12) that still gives at
// least three tiles for every four compute units, and a packed in-tile time
// of at most kTimeBits bits. Larger tiles cut fewer units and table phases;
// one tile per compute unit already keeps the chip busy (one 1024-thread
// workgroup fills a compute unit).
int auto_tile_log2(int64_t n_bins, int r_bits, int n_cu) {
  const int64_t min_tiles = std::max<int64_t>(1, 3 * (int64_t)n_cu / 4);
  int lb = 0;
  while (lb < 12 && (n_bins >> (lb + 1)) >= min_tiles) ++lb;
  lb = std::max(lb, 4);
  return std::min(lb, kTimeBits - r_bits);
}

size_t lib_lds_bytes(gtp_ctx c) { return (size_t)c->lds_words * 4; }

// LDS of the packed kernels: the library's meta + leakage prefix (rounded to
// 16 bytes), a tile of bins, and for the forward with table phases two slots.
size_t ml_lds_bytes(gtp_ctx c) {
  return packed_bins_word_offset(4 * c->n_cells + c->n_leak + 2 * c->n_cells * c->n_load) * 4;
}
size_t packed_lds_bytes(gtp_ctx c, int tile_log2) { return ml_lds_bytes(c) + ((size_t)16 << tile_log2); }
constexpr size_t kMaxLds = 160 * 1024;

// static LDS of the batched kernel (its work-item slot), kept out of the
// dynamic budget
constexpr size_t kBatchStaticLds = 64;

// Quads of one table slot for tiles of 2^tile_log2 bins: two slots fill what
// the bins and the library prefix leave of the LDS (the batched kernel's
// static slot included), a multiple of 64 quads, at most 4096; 0 (no table
// phases) below 256.
constexpr int32_t kMaxSlotQuads = 4096;
int32_t slot_quads_for(gtp_ctx c, int tile_log2) {
  const int64_t room = (int64_t)kMaxLds - (int64_t)kBatchStaticLds - (int64_t)packed_lds_bytes(c, tile_log2);
  const int64_t q = std::min<int64_t>(room / 32 / 64 * 64, kMaxSlotQuads);
  return q >= 256 ? (int32_t)q : 0;
}
size_t slot_bytes(int32_t slot_quads) { return 2 * (size_t)slot_quads * 16; }
// Longest unit of the packed layout by default; kernels hold a group's events
// in registers, 8 or 16 slots per lane. With 16 slots, workgroups of at most
// 512 threads (the registers of 1024 threads do not fit).
constexpr int kDefaultUnitEvents = 8;
constexpr int kXcds = 8;   // XCDs of the MI355X: workgroup i runs on XCD i % 8
constexpr int64_t kMaxFwdGrid = 1 << 20;   // workgroups of a packed forward launch (tiles beyond are strided)
int threads_for_slots(int th, int slots) { return (slots == 16 && th > 512) ? 512 : th; }
int unit_events_of(gtp_ctx c) { return c->tun.unit_events ? c->tun.unit_events : kDefaultUnitEvents; }
int slots_of(gtp_ctx c) { return unit_events_of(c) <= 8 ? 8 : 16; }


template <class K>
hipError_t lds_limit(K kern, size_t static_lds = 0) {
  return hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)(kMaxLds - static_lds));
}

template <int TH, int SL, bool SO, bool GL>
hipError_t lds_limits_one() {
  hipError_t e1 = lds_limit(k_fwd_packed<TH, SL, SO, GL>);
  hipError_t e2 = lds_limit(k_fwd_batched<TH, SL, SO, GL>, kBatchStaticLds);
  return e1 != hipSuccess ? e1 : e2;
}

template <bool GL>
hipError_t lds_limits_gl() {
  const hipError_t r[] = {lds_limits_one<256, 8, false, GL>(),  lds_limits_one<512, 8, false, GL>(),
                          lds_limits_one<1024, 8, false, GL>(), lds_limits_one<256, 16, false, GL>(),
                          lds_limits_one<512, 16, false, GL>(), lds_limits_one<256, 8, true, GL>(),
                          lds_limits_one<512, 8, true, GL>(),   lds_limits_one<1024, 8, true, GL>(),
                          lds_limits_one<256, 16, true, GL>(),  lds_limits_one<512, 16, true, GL>(),
                          lds_limit(k_adjoint_packed<1024, 8, GL, false>), lds_limit(k_adjoint_packed<512, 16, GL, false>),
                          lds_limit(k_adjoint_packed<1024, 8, GL, true>), lds_limit(k_adjoint_packed<512, 16, GL, true>)};
  for (hipError_t x : r)
    if (x != hipSuccess) return x;
  return hipSuccess;
}

hipError_t set_packed_lds_limits() {
  const hipError_t e = lds_limits_gl<false>();
  return e != hipSuccess ? e : lds_limits_gl<true>();
}

void drop_batch_packs(gtp_ctx c);
void drop_batch(gtp_ctx c);

void drop_pack(gtp_ctx c) {
  if (c->pk.ev || c->pk.gperm || c->pk_adj.ev || c->pk_adj.gperm) (void)hipStreamSynchronize(c->stream);
  if (c->pk.ev || c->pk.gperm) {
    c->dev_bytes -= c->pk.bytes;
    pack_free(&c->pk);
  }
  if (c->pk_adj.ev || c->pk_adj.gperm) {
    c->dev_bytes -= c->pk_adj.bytes;
    pack_free(&c->pk_adj);
  }
  c->pack_ok = false;
  c->pack_adj_ok = false;
  c->adj_ok = false;
}

EvView ev_view_of(gtp_ctx c, const gtp_events& ev) {
  EvView E;
  E.t = ev.t_ps;
  E.pb = ev.pin_bit;
  E.slew = ev.slew_ps;
  E.gate_off = ev.gate_off;
  E.n = ev.n_events;
  E.n_gates = c->n_gates;
  return E;
}

// Bin layout of an event window under the ctx parameters.
BinSpec bins_for(gtp_ctx c, int64_t t_end) {
  BinSpec B = c->bins;
  B.t_end = t_end;
  B.n_bins = (t_end + B.D - 1) / B.D;
  B.t32 = (t_end <= ((int64_t)1 << 32)) ? 1 : 0;
  B.n_tiles = 0;
  return B;
}

// Fixed-point exponent of a packed event set: the largest m <= 40 for which no
// bin can overflow (gtp_fixed_point_bits). Bounds: per event |energy| <=
// max|T| * (|1-alpha|+|alpha|)_max * (|1-beta|+|beta|)_max + load_cap * V^2
// (loads are limited to [0, load_cap] by the gate-record kernels), per bin at
// most max_bin_events events, and a total leakage rate below r_bound.
gtp_status choose_mfix(gtp_ctx c, const PackOut& pk, int64_t bin_ps, int32_t* m) {
  gtp_range r;
  r.max_bin_events = pk.max_bin_events;
  r.bin_ps = bin_ps;
  const double v2 = c->par.vdd * c->par.vdd;
  r.event_energy_fj = c->lib_tmax * (double)pk.alpha_span * c->beta_span +
                      c->load_cap * v2 * (c->par.sw_mode ? 1.0 : 0.5);
  r.leak_rate_fj_per_ps = c->r_bound;
  r.leak_value_nw = (double)GTP_MAX_LEAK_SCALE * c->lib_leak_max;
  const gtp_status st = gtp_fixed_point_bits(&r, m);
  if (st != GTP_OK)
    return fail(c, st,
                "bins of %lld ps with up to %lld events each exceed the fixed-point range (event energy bound %.3g fJ, "
                "leakage rate bound %.3g fJ/ps)",
                (long long)bin_ps, (long long)pk.max_bin_events, r.event_energy_fj, r.leak_rate_fj_per_ps);
  return GTP_OK;
}

// Packed layout of one event set (plan_buf: its gate-major lane-block plan);
// sets B.tile_log2 / B.n_tiles.
gtp_status pack_for(gtp_ctx c, const gtp_events& ev, const DevBuf& plan_buf, BinSpec& B, PackOut& pk, double& pack_ms,
                    int32_t* dbg_state = nullptr, int64_t* dbg_bin = nullptr,
                    const std::vector<int64_t>* gate_weight = nullptr, Workspace* arena = nullptr,
                    bool time_order = false) {
  if (B.r_bits > kTimeBits) return fail(c, GTP_ERR_UNSUPPORTED, "bin width above 2^%d ps", kTimeBits);
  int lb = c->tun.bins_per_tile_log2 ? c->tun.bins_per_tile_log2 : auto_tile_log2(B.n_bins, B.r_bits, c->n_cu);
  if (lb + B.r_bits > kTimeBits)
    return fail(c, GTP_ERR_UNSUPPORTED, "tile of 2^%d bins with %d-bit in-bin offsets exceeds %d bits", lb, B.r_bits,
                kTimeBits);
  if (packed_lds_bytes(c, lb) > kMaxLds)
    return fail(c, GTP_ERR_UNSUPPORTED, "tile of 2^%d bins and the library image exceed the LDS", lb);
  const int64_t nt = (B.n_bins + (1ll << lb) - 1) >> lb;
  if (nt >= (int64_t)INT32_MAX / 2) return fail(c, GTP_ERR_UNSUPPORTED, "%lld time tiles", (long long)nt);
  if (ev.n_events >= (int64_t)UINT32_MAX) return fail(c, GTP_ERR_UNSUPPORTED, "2^32 or more events in one trace");
  if (c->n_gates >= (1ll << 28) - 1) return fail(c, GTP_ERR_UNSUPPORTED, "2^28 or more gates");
  B.tile_log2 = lb;
  B.n_tiles = (int32_t)nt;
  PackIn in;
  in.ev = ev_view_of(c, ev);
  in.plan_blk = reinterpret_cast<const uint2*>(plan_buf.p);
  in.gate_cell = ptr<int32_t>(c->gate_cell);
  in.gate_init = ptr<uint32_t>(c->gate_init);
  in.gate_out = ptr<int32_t>(c->gate_out);
  in.h_gate_cell = c->h_gate_cell;
  in.n_in = c->h_nin;
  in.lib = lib_view(c);
  in.dbg_state = dbg_state;
  in.dbg_bin = dbg_bin;
  in.cq_lo = c->h_cq_lo;
  in.cq_hi = c->h_cq_hi;
  if (gate_weight) in.gate_weight = *gate_weight;
  in.slot_quads = slot_quads_for(c, lb);
  in.unit_events = unit_events_of(c);
  in.gate_block_log2 = c->tun.gate_block_log2 ? c->tun.gate_block_log2 : kGateBlockLog2;
  in.bins = B;
  in.stream = c->stream;
  in.ws = c->pk_ws;
  in.glitch_clk = c->par.glitch_clk_ps;
  in.arena = arena;
  in.time_order = time_order;
  const size_t ws_before = c->pk_ws[0].bytes + c->pk_ws[1].bytes;
  char msg[256] = {0};
  hipEvent_t e0 = nullptr, e1 = nullptr;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  if (e0) (void)hipEventRecord(e0, c->stream);
  const hipError_t st = pack_events(in, &pk, msg, sizeof msg);
  c->dev_bytes += (int64_t)(c->pk_ws[0].bytes + c->pk_ws[1].bytes) - (int64_t)ws_before;
  if (st != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    return fail(c, st == hipErrorOutOfMemory ? GTP_ERR_OUT_OF_MEMORY : GTP_ERR_HIP, "%s", msg);
  }
  if (e0 && e1) {
    float ms = 0.f;
    (void)hipEventRecord(e1, c->stream);
    (void)hipEventSynchronize(e1);
    (void)hipEventElapsedTime(&ms, e0, e1);
    pack_ms = ms;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  c->dev_bytes += pk.bytes;
  const gtp_status ms = choose_mfix(c, pk, B.D, &pk.mfix);
  if (ms != GTP_OK) {
    c->dev_bytes -= pk.bytes;
    pack_free(&pk);
    return ms;
  }
  return GTP_OK;
}

// The single-trace layout's output arrays come from an arena sized by the
// largest earlier layout, so rebuilding the layout (new events, or the next
// window of a stream) allocates and frees nothing once it has grown; the
// arena is grown only here, after drop_pack has waited for every kernel that
// read the previous layout.
gtp_status grow_pack_arena(gtp_ctx c) {
  if (c->pk_arena_want <= c->pk_arena.bytes) return GTP_OK;
  const size_t want = c->pk_arena_want + c->pk_arena_want / 8;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (c->pk_arena.p) (void)hipFree(c->pk_arena.p);
  c->dev_bytes -= (int64_t)c->pk_arena.bytes;
  c->pk_arena = Workspace{nullptr, 0};
  if (hipMalloc(&c->pk_arena.p, want) != hipSuccess) {
    (void)hipGetLastError();
    c->pk_arena = Workspace{nullptr, 0};
    c->pk_arena_want = 0;   // fall back to per-array allocations
    return GTP_OK;
  }
  c->pk_arena.bytes = want;
  c->dev_bytes += (int64_t)want;
  return GTP_OK;
}

gtp_status build_pack(gtp_ctx c) {
  if (c->pack_ok) return GTP_OK;
  drop_pack(c);
  TRY(grow_pack_arena(c));
  TRY(pack_for(c, c->ev, c->plan_blk, c->bins, c->pk, c->pack_ms, nullptr, nullptr, nullptr, &c->pk_arena));
  c->pk_arena_want = std::max(c->pk_arena_want, c->pk.need_bytes);
  c->pack_ok = true;
  return GTP_OK;
}

// The adjoint's layout: the same units, groups and gate order as the
// forward's, but inside a run of one (tile, gate block, length) the units are
// ordered by the time of their first event, so a group's bin-weight gathers
// fall in fewer cache lines (the forward keeps gate order: its gate-record
// gathers prefer it). Built once per layout, on the first adjoint; when it
// cannot be built (gate blocks above 2^16 gates, or no memory for it) the
// adjoint reads the forward's layout.
gtp_status build_pack_adj(gtp_ctx c) {
  if (c->pack_adj_ok) return GTP_OK;
  const int gbl = c->tun.gate_block_log2 ? c->tun.gate_block_log2 : kGateBlockLog2;
  if (gbl > 16) return GTP_OK;
  BinSpec B = c->bins;
  double ms = 0.0;
  if (pack_for(c, c->ev, c->plan_blk, B, c->pk_adj, ms, nullptr, nullptr, nullptr, nullptr, true) != GTP_OK) {
    if (c->pk_adj.ev || c->pk_adj.gperm) {
      c->dev_bytes -= c->pk_adj.bytes;
      pack_free(&c->pk_adj);
    }
    return GTP_OK;   // the forward's layout serves
  }
  c->pack_adj_ok = true;
  return GTP_OK;
}

const PackOut& adj_pack(gtp_ctx c) { return c->pack_adj_ok ? c->pk_adj : c->pk; }

// LDS of the packed adjoint: the library prefix, one cell's table quads (as
// many as fit, at most one slot), two FP64 accumulators per gate of the
// largest gate block.
constexpr int64_t kAdjAccBytes = 16;   // per gate: load and leakage-scale gradient (FP64)
int32_t adj_slot_quads(gtp_ctx c, int32_t max_gb) {
  const int64_t room = (int64_t)kMaxLds - (int64_t)ml_lds_bytes(c) - kAdjAccBytes * (int64_t)max_gb;
  return (int32_t)std::max<int64_t>(0, std::min<int64_t>(room / 16, kMaxSlotQuads));
}
size_t adj_lds_bytes(gtp_ctx c, int32_t max_gb) {
  return ml_lds_bytes(c) + 16 * (size_t)adj_slot_quads(c, max_gb) + (size_t)max_gb * kAdjAccBytes;
}

// Work items of the packed adjoint. Entries list, gate block by gate block
// and tile by tile, the groups holding the block's units with the lane range
// of those units; an item is one block's entries over one of the tile ranges
// shared by all blocks (about three items per CU in all).
gtp_status adj_plan(gtp_ctx c) {
  if (c->adj_ok) return GTP_OK;
  const PackOut& pk = adj_pack(c);
  const int32_t n_gb = pk.n_gb, n_tiles = c->bins.n_tiles;
  const int64_t n_reg = (int64_t)n_tiles * n_gb;
  if (pk.n_groups >= ((int64_t)1 << 31)) return fail(c, GTP_ERR_UNSUPPORTED, "too many groups for the adjoint");
  std::vector<uint32_t> rf((size_t)n_reg + 1), tf((size_t)n_tiles + 1);
  std::vector<int32_t> tg((size_t)n_tiles + 1);
  HIPCHK(c, hipMemcpyAsync(rf.data(), pk.reg_first, rf.size() * 4, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(tf.data(), pk.tfirst, tf.size() * 4, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(tg.data(), pk.tile_grp, tg.size() * 4, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  int32_t max_gb = 0;
  for (int32_t g = 0; g < n_gb; ++g) max_gb = std::max(max_gb, pk.h_gb_start[g + 1] - pk.h_gb_start[g]);
  int64_t total = 0;
  for (int64_t e : pk.h_reg_events) total += e;
  // tile ranges shared by every gate block, about three items per CU in all
  int32_t active_gb = 0;
  for (int32_t g = 0; g < n_gb; ++g) {
    int64_t e = 0;
    for (int32_t k = 0; k < n_tiles; ++k) e += pk.h_reg_events[(size_t)k * n_gb + g];
    if (e > 0) ++active_gb;
  }
  const int64_t want = 3 * (int64_t)std::max(c->n_cu, 1);
  int64_t nr = (want + std::max(active_gb, 1) - 1) / std::max(active_gb, 1);
  nr = (nr + kXcds - 1) / kXcds * kXcds;  // a multiple of the XCD count
  const int32_t n_rng = (int32_t)std::max<int64_t>(1, std::min<int64_t>(n_tiles, nr));
  const int32_t rng_tiles = (n_tiles + n_rng - 1) / n_rng;
  struct Item { int64_t ev; int32_t gb, rng; int64_t e0, e1; };
  std::vector<Item> items;
  std::vector<int4> ent;
  for (int32_t g = 0; g < n_gb; ++g) {
    for (int32_t k0 = 0; k0 < n_tiles; k0 += rng_tiles) {
      const int64_t e0 = (int64_t)ent.size();
      int64_t acc = 0;
      for (int32_t k = k0; k < std::min(n_tiles, k0 + rng_tiles); ++k) {
        const int64_t r = (int64_t)k * n_gb + g;
        const int64_t j0 = rf[r], j1 = rf[r + 1];
        if (j0 >= j1) continue;
        const int64_t t0 = tf[k];
        for (int64_t q = (j0 - t0) / kGroupUnits; q <= (j1 - 1 - t0) / kGroupUnits; ++q) {
          const int64_t u0 = t0 + q * kGroupUnits;
          const int lo = (int)std::max<int64_t>(j0 - u0, 0), hi = (int)std::min<int64_t>(j1 - u0, kGroupUnits);
          ent.push_back(make_int4((int32_t)(tg[k] + q), k, lo | (hi << 8), 0));
        }
        acc += pk.h_reg_events[(size_t)r];
      }
      if ((int64_t)ent.size() > e0) items.push_back({acc, g, k0 / rng_tiles, e0, (int64_t)ent.size()});
    }
  }
  if ((int64_t)ent.size() >= ((int64_t)1 << 31)) return fail(c, GTP_ERR_UNSUPPORTED, "too many adjoint entries");
  // rows of the partial table: a block's items get consecutive rows
  std::vector<int64_t> gb_row((size_t)n_gb, 0);
  std::vector<int32_t> gb_rows((size_t)n_gb, 0);
  std::vector<AdjItem> h(std::max<size_t>(items.size(), 1));
  int64_t rows = 0;
  bool tab_only = true;   // every item's table slot holds all of its cell's quads
  for (size_t i = 0; i < items.size(); ++i) {
    const int32_t g = items[i].gb;
    const int64_t ng = pk.h_gb_start[g + 1] - pk.h_gb_start[g];
    if (gb_rows[g] == 0) gb_row[g] = rows;
    const int32_t cell = pk.h_gb_cell[g];
    const int32_t qn = std::min(c->h_cq_hi[cell] - c->h_cq_lo[cell], adj_slot_quads(c, max_gb));
    if (qn < c->h_cq_hi[cell] - c->h_cq_lo[cell]) tab_only = false;
    h[i] = AdjItem{g, (int32_t)items[i].e0, (int32_t)items[i].e1, c->h_cq_lo[cell], gb_row[g] + gb_rows[g] * ng, qn, 0};
    gb_rows[g]++;
    rows += ng;
  }
  // launch order: workgroup i runs on XCD i % kXcds, and tile range r is
  // given to XCD r % kXcds, taken range by range (largest items first within
  // a range): the items resident on one XCD read the bin weights of about one
  // tile range, which then stays in that XCD's L2. Empty items pad the
  // interleave where one XCD has fewer items than another.
  std::vector<std::vector<int32_t>> per((size_t)kXcds);
  for (size_t i = 0; i < items.size(); ++i) per[(size_t)(items[i].rng % kXcds)].push_back((int32_t)i);
  size_t longest = 0;
  for (auto& v : per) {
    std::stable_sort(v.begin(), v.end(), [&](int32_t a, int32_t b) {
      if (items[a].rng != items[b].rng) return items[a].rng < items[b].rng;
      return items[a].ev > items[b].ev;
    });
    longest = std::max(longest, v.size());
  }
  const AdjItem pad{0, 0, 0, 0, -1, 0, 0};
  std::vector<AdjItem> hs;
  for (size_t j = 0; j < longest; ++j)
    for (int x = 0; x < kXcds; ++x) hs.push_back(j < per[(size_t)x].size() ? h[(size_t)per[(size_t)x][j]] : pad);
  while (!hs.empty() && hs.back().row < 0) hs.pop_back();
  if (hs.empty()) hs.push_back(pad);
  if (ent.empty()) ent.push_back(make_int4(0, 0, 0, 0));
  TRY(ensure(c, c->adj_items, hs.size() * sizeof(AdjItem)));
  TRY(ensure(c, c->adj_entries, ent.size() * sizeof(int4)));
  TRY(ensure(c, c->adj_gbs, pk.h_gb_start.size() * 4));
  TRY(ensure(c, c->adj_gbrow, gb_row.size() * 8));
  TRY(ensure(c, c->adj_gbrows, gb_rows.size() * 4));
  TRY(ensure(c, c->adj_part, (size_t)std::max<int64_t>(rows, 1) * sizeof(double2)));
  HIPCHK(c, hipMemcpyAsync(c->adj_items.p, hs.data(), hs.size() * sizeof(AdjItem), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->adj_entries.p, ent.data(), ent.size() * sizeof(int4), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->adj_gbs.p, pk.h_gb_start.data(), pk.h_gb_start.size() * 4, hipMemcpyHostToDevice,
                           c->stream));
  HIPCHK(c, hipMemcpyAsync(c->adj_gbrow.p, gb_row.data(), gb_row.size() * 8, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->adj_gbrows.p, gb_rows.data(), gb_rows.size() * 4, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->adj_n_items = items.empty() ? 0 : (int64_t)hs.size();
  c->adj_max_gb = max_gb;
  c->adj_tab_only = tab_only;
  c->adj_ok = true;
  return GTP_OK;
}

gtp_status gate_prep(gtp_ctx c, const float* net_load, const float* leak_scale, int32_t m) {
  TRY(ensure(c, c->gprep, (size_t)std::max<int64_t>(c->n_gates, 1) * sizeof(GatePrep)));
  TRY(ensure(c, c->L0, 8));
  TRY(fill_u64(c, c->L0.p, 1, 0ull));
  if (c->n_gates == 0) return GTP_OK;
  PrepArgs a;
  const LibView L = lib_view(c);
  a.gate_cell = ptr<int32_t>(c->gate_cell);
  a.gate_out = ptr<int32_t>(c->gate_out);
  a.gate_init = ptr<uint32_t>(c->gate_init);
  a.net_load = net_load;
  a.leak_scale = leak_scale;
  a.meta = L.meta;
  a.leak = L.leak;
  a.wide = L.wide;
  a.load = ptr<float>(c->load_axis);
  a.load_inv = ptr<float>(c->load_inv);
  a.n_load = c->n_load;
  a.n_gates = c->n_gates;
  a.vdd = c->par.vdd;
  a.sw_mode = c->par.sw_mode;
  a.rate_scale = rate_scale_of(m);
  a.max_scale = GTP_MAX_LEAK_SCALE;
  a.load_cap = (float)c->load_cap;
  a.all_pins = c->all_pins;
  a.out = ptr<GatePrep>(c->gprep);
  a.L0 = ptr<unsigned long long>(c->L0);
  a.flag = ptr<int32_t>(c->flag);
  LAUNCH(c, "k_gate_prep", k_gate_prep, dim3(grid_for(c->n_gates, 256)), dim3(256), 0, a);
  return GTP_OK;
}

}  // namespace

// ============================================================================
// C ABI
// ============================================================================
extern "C" {

gtp_status gtp_fixed_point_bits(const gtp_range* r, int32_t* m_out) {
  if (!r || !m_out || r->max_bin_events < 0 || r->bin_ps < 1 || !(r->event_energy_fj >= 0.0) ||
      !(r->leak_rate_fj_per_ps >= 0.0) || !(r->leak_value_nw >= 0.0) || !std::isfinite(r->event_energy_fj) ||
      !std::isfinite(r->leak_rate_fj_per_ps) || !std::isfinite(r->leak_value_nw))
    return GTP_ERR_INVALID_ARG;
  const double bound = (double)r->max_bin_events * r->event_energy_fj + (double)r->bin_ps * r->leak_rate_fj_per_ps;
  int m = kMaxMfix;
  // the largest m with 2^m * bound < 2^62 (2x margin for the sum of the
  // terms and the FP64 evaluation) and a quantised rate below 2^30
  while (m >= kMinMfix && (std::ldexp(bound, m) >= std::ldexp(1.0, 62) ||
                           std::ldexp(r->leak_value_nw * 1e-6, m) >= std::ldexp(1.0, 30)))
    --m;
  if (m < kMinMfix) return GTP_ERR_UNSUPPORTED;
  *m_out = m;
  return GTP_OK;
}

gtp_status gtp_expand_when(int32_t n_pins, int32_t n_patterns, const uint32_t* care, const uint32_t* value,
                           const int32_t* item, int32_t default_item, int32_t* out) {
  if (n_pins < 0 || n_pins > kSiplMaxPins || n_patterns < 0 || !out ||
      (n_patterns > 0 && (!care || !value || !item)))
    return GTP_ERR_INVALID_ARG;
  const uint32_t full = (1u << n_pins) - 1u;
  for (int32_t k = 0; k < n_patterns; ++k)
    if (care[k] & ~full) return GTP_ERR_INVALID_ARG;
  const int64_t n = 1ll << n_pins;
  std::vector<uint8_t> done((size_t)n, 0);
  // patterns in order; every assignment of a pattern's don't-care pins
  // (the submasks of its free pins) names one entry, which keeps the item of
  // the first pattern that reached it
  for (int32_t k = 0; k < n_patterns; ++k) {
    const uint32_t fixed = value[k] & care[k], free_pins = full & ~care[k];
    uint32_t sub = free_pins;
    for (;;) {
      const uint32_t s = fixed | sub;
      if (!done[s]) {
        done[s] = 1;
        out[s] = item[k];
      }
      if (sub == 0) break;
      sub = (sub - 1u) & free_pins;
    }
  }
  for (int64_t s = 0; s < n; ++s)
    if (!done[(size_t)s]) out[s] = default_item;
  return GTP_OK;
}

gtp_status gtp_create(gtp_ctx* out, int hip_device, void* hip_stream) {
  if (!out) return GTP_ERR_INVALID_ARG;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || hip_device < 0 || hip_device >= n) {
    (void)hipGetLastError();
    return GTP_ERR_INVALID_ARG;
  }
  gtp_ctx c = new (std::nothrow) gtp_ctx_s();
  if (!c) return GTP_ERR_OUT_OF_MEMORY;
  c->dev = hip_device;
  {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, hip_device) == hipSuccess && cus > 0)
      c->n_cu = cus;
    hipDeviceProp_t pr;
    if (hipGetDeviceProperties(&pr, hip_device) == hipSuccess) c->dev_total = pr.totalGlobalMem;
    (void)hipGetLastError();
  }
  c->stream = (hipStream_t)hip_stream;
  if (hipSetDevice(hip_device) != hipSuccess) {
    delete c;
    return GTP_ERR_HIP;
  }
  if (scratch_address(hip_device, &c->scratch_dev) != hipSuccess) {
    (void)hipGetLastError();
    delete c;
    return GTP_ERR_HIP;
  }
  if (ensure(c, c->flag, 256) != GTP_OK || ensure(c, c->first_bad, 256) != GTP_OK) {
    delete c;
    return GTP_ERR_OUT_OF_MEMORY;
  }
  // dynamic LDS above the 64 KB default: library image plus a tile of bins
  if (set_packed_lds_limits() != hipSuccess) {
    (void)hipGetLastError();
    delete c;
    return GTP_ERR_HIP;
  }
  if (fill_u64(c, c->flag.p, 1, 0ull) != GTP_OK) {
    delete c;
    return GTP_ERR_HIP;
  }
  *out = c;
  return GTP_OK;
}

gtp_status gtp_destroy(gtp_ctx c) {
  if (!c) return GTP_OK;
  (void)hipSetDevice(c->dev);
  (void)hipStreamSynchronize(c->stream);
  drop_pack(c);
  drop_batch(c);
  for (Workspace& w : c->pk_ws)
    if (w.p) (void)hipFree(w.p);
  if (c->pk_arena.p) (void)hipFree(c->pk_arena.p);
  if (c->copy_stream) (void)hipStreamSynchronize(c->copy_stream);
  for (auto& sl : c->st_slot) {
    for (DevBuf* b : {&sl.gate_off, &sl.t, &sl.pb, &sl.slew}) release(c, *b);
    if (sl.copied) (void)hipEventDestroy(sl.copied);
    if (sl.done) (void)hipEventDestroy(sl.done);
  }
  release(c, c->st_init);
  if (c->copy_stream) (void)hipStreamDestroy(c->copy_stream);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  DevBuf* all[] = {&c->lib_img, &c->load_axis, &c->load_inv, &c->quads, &c->wide_cell, &c->wide_pat, &c->wide_sipl,
                   &c->gate_cell, &c->gate_out,
                   &c->gate_init, &c->plan_blk, &c->blk_tmp, &c->blk_tmp2, &c->scan_sums, &c->gprep, &c->gparam, &c->l0_part, &c->tile_tot, &c->tile_base,
                   &c->X, &c->S, &c->exS, &c->L0, &c->flag, &c->first_bad, &c->adj_w, &c->adj_c, &c->adj_exc,
                   &c->adj_wg, &c->adj_gtile, &c->adj_total, &c->rep_small, &c->gC, &c->gL, &c->adj_items, &c->adj_entries, &c->adj_gbs, &c->adj_gbrow, &c->adj_gbrows, &c->adj_part, &c->b_tab, &c->b_items,
                   &c->b_fin, &c->b_X, &c->b_S, &c->b_tile_tot, &c->b_tile_base, &c->tun_in, &c->tun_out};
  for (DevBuf* b : all) release(c, *b);
  prof_clear(c);
  for (hipEvent_t e : c->prof_pool) (void)hipEventDestroy(e);
  delete c;
  return GTP_OK;
}

gtp_status gtp_set_stream(gtp_ctx c, void* s) {
  if (!c) return GTP_ERR_INVALID_ARG;
  c->stream = (hipStream_t)s;
  return GTP_OK;
}

const char* gtp_last_error(gtp_ctx c) { return c ? c->err.c_str() : "null context"; }

int64_t gtp_bad_event(gtp_ctx c) { return c ? c->bad_event : -1; }

int64_t gtp_device_bytes(gtp_ctx c) { return c ? c->dev_bytes : 0; }

gtp_status gtp_sync(gtp_ctx c) {
  if (!c) return GTP_ERR_INVALID_ARG;
  HIPCHK(c, hipSetDevice(c->dev));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  int32_t flag = 0;
  HIPCHK(c, hipMemcpy(&flag, c->flag.p, 4, hipMemcpyDeviceToHost));
  if (flag) {
    fill_u64(c, c->flag.p, 1, 0ull);
    (void)hipStreamSynchronize(c->stream);
    if (flag & 2)
      return fail(c, GTP_ERR_LOAD_RANGE, "a net load was negative, not finite or above %g fF (used as 0)",
                  c->load_cap);
    return fail(c, GTP_ERR_SCALE_RANGE, "a leakage scale was negative, not finite or above %g (used as 0)",
                (double)GTP_MAX_LEAK_SCALE);
  }
  return GTP_OK;
}

gtp_status gtp_load_library(gtp_ctx c, const gtp_library* lib) {
  if (!c || !lib) return GTP_ERR_INVALID_ARG;
  HIPCHK(c, hipSetDevice(c->dev));
  const int nc = lib->n_cells, ns = lib->n_slew, nl = lib->n_load;
  if (nc <= 0 || ns < 2 || ns > 16 || nl < 2 || nl > 16)
    return fail(c, GTP_ERR_INVALID_ARG, "library sizes n_cells=%d n_slew=%d n_load=%d", nc, ns, nl);
  if (!lib->n_inputs || !lib->slew_axis_ps || !lib->load_axis_ff || !lib->table_base || !lib->tables_fj)
    return fail(c, GTP_ERR_INVALID_ARG, "null library array");
  if (lib->n_tables <= 0) return fail(c, GTP_ERR_INVALID_ARG, "library without tables");
  const int64_t Q = (int64_t)(ns - 1) * (nl - 1);
  if (lib->n_tables * Q >= (int64_t)INT32_MAX) return fail(c, GTP_ERR_UNSUPPORTED, "tables too large");
  std::vector<CellMeta> meta(nc);
  std::vector<int32_t> cq_lo(nc), cq_hi(nc);   // quads of each cell's tables
  std::vector<int32_t> mapq;
  std::vector<float> leak;
  std::vector<double> cell_leak_max(nc, 0.0);
  float leak_max = 0.f;
  if (lib->all_pin_state != 0 && lib->all_pin_state != 1)
    return fail(c, GTP_ERR_INVALID_ARG, "all_pin_state %d (0 or 1)", lib->all_pin_state);
  const int allp = lib->all_pin_state;
  const bool pats = lib->n_tpat != nullptr;
  if (pats && (!lib->tpat_base || !lib->tpat_care || !lib->tpat_value || !lib->tpat_table || !lib->n_lpat ||
               !lib->lpat_base || !lib->lpat_care || !lib->lpat_value || !lib->lpat_leak_nw ||
               lib->n_tpat_total < 0 || lib->n_lpat_total < 0))
    return fail(c, GTP_ERR_INVALID_ARG, "null or negative-length state-pattern array");
  std::vector<WideCell> wcell((size_t)nc, WideCell{0, 0, 0, 0, 0, 0});
  std::vector<uint2> wpat;
  std::vector<uint8_t> wsipl;
  bool has_wide = false;
  for (int cc = 0; cc < nc; ++cc) {
    const int I = lib->n_inputs[cc];
    const bool by_pat = pats && lib->n_tpat[cc] > 0;
    const int nsp = I + allp;   // state pins
    if (!by_pat && (I < 1 || nsp > 8))
      return fail(c, GTP_ERR_UNSUPPORTED, "cell %d: %d inputs given as per-state arrays (1..%d; wider cells need "
                  "state patterns)", cc, I, 8 - allp);
    if (by_pat && (I < 1 || I > 31))
      return fail(c, GTP_ERR_UNSUPPORTED, "cell %d has %d inputs (supported 1..31)", cc, I);
    const int64_t tb = lib->table_base[cc];
    if (tb < 0 || tb >= lib->n_tables) return fail(c, GTP_ERR_INVALID_ARG, "cell %d: table base out of range", cc);
    for (int i = 0; i + 1 < ns; ++i)
      if (!(lib->slew_axis_ps[cc * ns + i] < lib->slew_axis_ps[cc * ns + i + 1]))
        return fail(c, GTP_ERR_INVALID_ARG, "cell %d: slew axis not strictly increasing", cc);
    for (int j = 0; j + 1 < nl; ++j)
      if (!(lib->load_axis_ff[cc * nl + j] < lib->load_axis_ff[cc * nl + j + 1]))
        return fail(c, GTP_ERR_INVALID_ARG, "cell %d: load axis not strictly increasing", cc);
    // the cell's map entries (local table ids, fall and rise per entry) and
    // leakage values: per state for a kCellDirect cell, per pattern otherwise
    std::vector<int64_t> tid;
    std::vector<float> lv;
    int16_t mode = kCellDirect;
    if (!by_pat) {
      if (!lib->map_base || !lib->state_to_table || !lib->leak_base || !lib->leak_nw)
        return fail(c, GTP_ERR_INVALID_ARG, "cell %d: null per-state array", cc);
      const int64_t nst = 1ll << nsp;
      const int64_t mb = lib->map_base[cc], lbs = lib->leak_base[cc];
      if (mb < 0 || mb + 2 * nst > lib->n_map || lbs < 0 || lbs + nst > lib->n_leak)
        return fail(c, GTP_ERR_INVALID_ARG, "cell %d: map/leak base out of range", cc);
      tid.assign(lib->state_to_table + mb, lib->state_to_table + mb + 2 * nst);
      lv.assign(lib->leak_nw + lbs, lib->leak_nw + lbs + nst);
    } else {
      const int64_t nt = lib->n_tpat[cc], nlp = lib->n_lpat[cc];
      const int64_t t0 = lib->tpat_base[cc], l0 = lib->lpat_base[cc];
      if (nt > 256 || nlp < 1 || nlp > 256)
        return fail(c, GTP_ERR_INVALID_ARG, "cell %d: %lld table and %lld leakage patterns (1..256 each)", cc,
                    (long long)nt, (long long)nlp);
      if (t0 < 0 || t0 + nt > lib->n_tpat_total || l0 < 0 || l0 + nlp > lib->n_lpat_total)
        return fail(c, GTP_ERR_INVALID_ARG, "cell %d: pattern base out of range", cc);
      const uint32_t smask = nsp >= 32 ? 0xffffffffu : (1u << nsp) - 1u;
      for (int64_t k = 0; k < nt; ++k)
        if (lib->tpat_care[t0 + k] & ~smask)
          return fail(c, GTP_ERR_INVALID_ARG, "cell %d: table pattern %lld names a pin outside the state", cc,
                      (long long)k);
      for (int64_t k = 0; k < nlp; ++k)
        if (lib->lpat_care[l0 + k] & ~smask)
          return fail(c, GTP_ERR_INVALID_ARG, "cell %d: leakage pattern %lld names a pin outside the state", cc,
                      (long long)k);
      if (lib->tpat_care[t0 + nt - 1] != 0u || lib->lpat_care[l0 + nlp - 1] != 0u)
        return fail(c, GTP_ERR_INVALID_ARG, "cell %d: the last pattern of each list must have no care pins", cc);
      if (nsp <= kSiplMaxPins) {
        // expand both lists into per-state pattern indices
        const int64_t nst = 1ll << nsp;
        std::vector<int32_t> idx((size_t)std::max(nt, nlp)), it((size_t)nst), il((size_t)nst);
        for (size_t k = 0; k < idx.size(); ++k) idx[k] = (int32_t)k;
        if (gtp_expand_when(nsp, (int32_t)nt, lib->tpat_care + t0, lib->tpat_value + t0, idx.data(),
                            (int32_t)nt - 1, it.data()) != GTP_OK ||
            gtp_expand_when(nsp, (int32_t)nlp, lib->lpat_care + l0, lib->lpat_value + l0, idx.data(),
                            (int32_t)nlp - 1, il.data()) != GTP_OK)
          return fail(c, GTP_ERR_INVALID_ARG, "cell %d: state patterns", cc);
        if (nsp <= 8) {
          for (int64_t st = 0; st < nst; ++st) {
            tid.push_back(lib->tpat_table[2 * (t0 + it[st])]);
            tid.push_back(lib->tpat_table[2 * (t0 + it[st]) + 1]);
            lv.push_back(lib->lpat_leak_nw[l0 + il[st]]);
          }
        } else {
          mode = kCellSipl;
          wcell[cc].t_sipl = (int64_t)wsipl.size();
          for (int64_t st = 0; st < nst; ++st) wsipl.push_back((uint8_t)it[st]);
          wcell[cc].l_sipl = (int64_t)wsipl.size();
          for (int64_t st = 0; st < nst; ++st) wsipl.push_back((uint8_t)il[st]);
        }
      } else {
        mode = kCellScan;
        wcell[cc].t_first = (int32_t)wpat.size();
        for (int64_t k = 0; k < nt; ++k) wpat.push_back(make_uint2(lib->tpat_care[t0 + k], lib->tpat_value[t0 + k]));
        wcell[cc].l_first = (int32_t)wpat.size();
        for (int64_t k = 0; k < nlp; ++k) wpat.push_back(make_uint2(lib->lpat_care[l0 + k], lib->lpat_value[l0 + k]));
      }
      if (mode != kCellDirect) {
        has_wide = true;
        wcell[cc].t_n = (int32_t)nt;
        wcell[cc].l_n = (int32_t)nlp;
        tid.assign(lib->tpat_table + 2 * t0, lib->tpat_table + 2 * (t0 + nt));
        lv.assign(lib->lpat_leak_nw + l0, lib->lpat_leak_nw + l0 + nlp);
      }
    }
    meta[cc].n_in = (int16_t)I;
    meta[cc].mode = mode;
    meta[cc].map_off = (int32_t)mapq.size();
    meta[cc].leak_off = (int32_t)leak.size();
    meta[cc].axis_off = cc * ns;
    int64_t t_lo = INT64_MAX, t_hi = -1;
    for (const int64_t k : tid) {
      if (k < 0 || tb + k >= lib->n_tables)
        return fail(c, GTP_ERR_INVALID_ARG, "cell %d: table id %lld out of range", cc, (long long)k);
      mapq.push_back((int32_t)((tb + k) * Q));
      t_lo = std::min(t_lo, tb + k);
      t_hi = std::max(t_hi, tb + k);
    }
    cq_lo[cc] = (int32_t)(t_lo * Q);
    cq_hi[cc] = (int32_t)((t_hi + 1) * Q);
    for (const float v : lv) {
      if (!(v >= 0.f) || !std::isfinite(v)) return fail(c, GTP_ERR_INVALID_ARG, "cell %d: bad leakage value", cc);
      leak.push_back(v);
      leak_max = std::max(leak_max, v);
      cell_leak_max[cc] = std::max(cell_leak_max[cc], (double)v);
    }
    if (mapq.size() >= (size_t)INT32_MAX / 2 || leak.size() >= (size_t)INT32_MAX / 2 || wpat.size() >= (size_t)INT32_MAX)
      return fail(c, GTP_ERR_UNSUPPORTED, "library too large");
  }
  for (int64_t i = 0; i < lib->n_tables * ns * nl; ++i)
    if (!std::isfinite(lib->tables_fj[i])) return fail(c, GTP_ERR_INVALID_ARG, "non-finite table entry %lld",
                                                       (long long)i);
  const int32_t n_map = (int32_t)mapq.size(), n_leak = (int32_t)leak.size();
  const int64_t words = 4ll * nc + n_leak + 2ll * nc * nl + n_map + 2ll * nc * ns;
  if (words * 4 > 48 * 1024)
    return fail(c, GTP_ERR_UNSUPPORTED, "library image of %lld bytes exceeds the 48 KB LDS budget",
                (long long)(words * 4));
  std::vector<uint32_t> img((size_t)words);
  memcpy(img.data(), meta.data(), sizeof(CellMeta) * nc);
  memcpy(img.data() + 4 * nc, leak.data(), 4 * (size_t)n_leak);
  float* load_img = reinterpret_cast<float*>(img.data() + 4 * nc + n_leak);
  float* load_inv_img = load_img + (size_t)nc * nl;
  memcpy(load_inv_img + (size_t)nc * nl, mapq.data(), 4 * (size_t)n_map);
  float* slew = reinterpret_cast<float*>(load_inv_img + (size_t)nc * nl + n_map);
  float* slew_inv = slew + (size_t)nc * ns;
  std::vector<float> load((size_t)nc * nl), load_inv((size_t)nc * nl, 0.f);
  for (int cc = 0; cc < nc; ++cc) {
    for (int i = 0; i < ns; ++i) {
      slew[cc * ns + i] = lib->slew_axis_ps[cc * ns + i];
      slew_inv[cc * ns + i] =
          (i + 1 < ns) ? (float)(1.0 / ((double)lib->slew_axis_ps[cc * ns + i + 1] - lib->slew_axis_ps[cc * ns + i]))
                       : 0.f;
    }
    for (int j = 0; j < nl; ++j) {
      load[cc * nl + j] = lib->load_axis_ff[cc * nl + j];
      load_inv[cc * nl + j] =
          (j + 1 < nl) ? (float)(1.0 / ((double)lib->load_axis_ff[cc * nl + j + 1] - lib->load_axis_ff[cc * nl + j]))
                       : 0.f;
    }
  }
  std::copy(load.begin(), load.end(), load_img);
  std::copy(load_inv.begin(), load_inv.end(), load_inv_img);
  // quads: (T[i][j], T[i][j+1], T[i+1][j], T[i+1][j+1]) per table and axis cell
  std::vector<float> quads((size_t)(lib->n_tables * Q * 4));
  for (int64_t T = 0; T < lib->n_tables; ++T) {
    const float* tb = lib->tables_fj + T * ns * nl;
    for (int i = 0; i + 1 < ns; ++i)
      for (int j = 0; j + 1 < nl; ++j) {
        float* q = &quads[(size_t)((T * Q + i * (nl - 1) + j) * 4)];
        q[0] = tb[i * nl + j];
        q[1] = tb[i * nl + j + 1];
        q[2] = tb[(i + 1) * nl + j];
        q[3] = tb[(i + 1) * nl + j + 1];
      }
  }
  if (has_wide) {
    TRY(ensure(c, c->wide_cell, wcell.size() * sizeof(WideCell)));
    TRY(ensure(c, c->wide_pat, std::max<size_t>(wpat.size(), 1) * sizeof(uint2)));
    TRY(ensure(c, c->wide_sipl, std::max<size_t>(wsipl.size(), 1)));
    HIPCHK(c, hipMemcpy(c->wide_cell.p, wcell.data(), wcell.size() * sizeof(WideCell), hipMemcpyHostToDevice));
    if (!wpat.empty())
      HIPCHK(c, hipMemcpy(c->wide_pat.p, wpat.data(), wpat.size() * sizeof(uint2), hipMemcpyHostToDevice));
    if (!wsipl.empty()) HIPCHK(c, hipMemcpy(c->wide_sipl.p, wsipl.data(), wsipl.size(), hipMemcpyHostToDevice));
  }
  TRY(ensure(c, c->lib_img, img.size() * 4));
  TRY(ensure(c, c->load_axis, load.size() * 4));
  TRY(ensure(c, c->load_inv, load_inv.size() * 4));
  TRY(ensure(c, c->quads, quads.size() * 4));
  HIPCHK(c, hipMemcpy(c->lib_img.p, img.data(), img.size() * 4, hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(c->load_axis.p, load.data(), load.size() * 4, hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(c->load_inv.p, load_inv.data(), load_inv.size() * 4, hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(c->quads.p, quads.data(), quads.size() * 4, hipMemcpyHostToDevice));
  c->n_cells = nc;
  c->n_slew = ns;
  c->n_load = nl;
  c->n_map = n_map;
  c->n_leak = n_leak;
  c->n_tables = lib->n_tables;
  c->all_pins = allp;
  c->has_wide = has_wide;
  c->lds_words = (int32_t)words;
  c->h_nin.assign(lib->n_inputs, lib->n_inputs + nc);
  c->h_cq_lo = cq_lo;
  c->h_cq_hi = cq_hi;
  // inputs of the fixed-point range (choose_mfix): largest |table entry|,
  // largest leakage value, the load limit (4x the largest load knot) and the
  // largest |1-beta|+|beta| of a load in [0, load_cap] (at one of the two
  // ends: beta is affine in the load on each axis segment)
  {
    double tmax = 0.0, lmax_axis = 0.0, span = 1.0;
    for (int64_t i = 0; i < lib->n_tables * ns * nl; ++i) tmax = std::max(tmax, std::fabs((double)lib->tables_fj[i]));
    for (int cc = 0; cc < nc; ++cc) lmax_axis = std::max(lmax_axis, (double)lib->load_axis_ff[cc * nl + nl - 1]);
    const double cap = 4.0 * std::max(lmax_axis, 1e-3);
    for (int cc = 0; cc < nc; ++cc) {
      const float* la = lib->load_axis_ff + cc * nl;
      for (double C : {0.0, cap}) {
        int j = 0;
        for (int m = 1; m < nl - 1; ++m) j += ((double)la[m] <= C) ? 1 : 0;
        const double b = (C - la[j]) / ((double)la[j + 1] - la[j]);
        span = std::max(span, std::fabs(1.0 - b) + std::fabs(b));
      }
    }
    c->lib_tmax = tmax;
    c->lib_leak_max = leak_max;
    c->load_cap = cap;
    c->beta_span = span;
    c->h_leak_max = cell_leak_max;
  }
  c->lib_ok = true;
  c->net_ok = false;
  c->ev_ok = false;
  drop_pack(c);
  drop_batch(c);
  return GTP_OK;
}

}  // extern "C"

namespace {
__global__ void k_check_netlist(const int32_t* cell, const int32_t* out, int64_t n, int32_t n_cells, int64_t n_nets,
                                int32_t* bad) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  if (cell[g] < 0 || cell[g] >= n_cells || out[g] < 0 || (int64_t)out[g] >= n_nets) atomicOr(bad, 1);
}
// Checks every event of ev (synchronises); the first offending event in
// gate-major order sets c->bad_event and the status.
gtp_status validate_events(gtp_ctx c, const gtp_events& ev, const DevBuf& plan, int64_t n_blocks) {
  if (n_blocks == 0) return GTP_OK;
  TRY(fill_u64(c, c->first_bad.p, 1, ~0ull));
  ValArgs a;
  a.ev = ev_view_of(c, ev);
  a.plan = reinterpret_cast<const uint2*>(plan.p);
  a.gate_cell = ptr<int32_t>(c->gate_cell);
  a.gate_init = ptr<uint32_t>(c->gate_init);
  a.meta = lib_view(c).meta;
  a.t_end = ev.t_end_ps;
  a.first = ptr<unsigned long long>(c->first_bad);
  LAUNCH(c, "k_validate", k_validate, dim3(grid_for(n_blocks, kFwdThreads)), dim3(kFwdThreads), 0, a);
  unsigned long long key = 0;
  HIPCHK(c, hipMemcpyAsync(&key, c->first_bad.p, 8, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (key != ~0ull) {
    const int code = (int)(key & 7);
    c->bad_event = (int64_t)(key >> 3);
    static const char* what[] = {"", "time outside [0, t_end)", "time decreases within its gate",
                                 "pin above the output pin", "pin repeated at one timestamp", "not a toggle"};
    const gtp_status st = (code == 1 || code == 3) ? GTP_ERR_EVENT_RANGE
                          : (code == 5)            ? GTP_ERR_NOT_TOGGLE
                                                   : GTP_ERR_EVENT_ORDER;
    return fail(c, st, "event %lld: %s", (long long)c->bad_event, what[code]);
  }
  return GTP_OK;
}

// Checks a caller's event descriptor against the netlist (synchronises).
gtp_status check_event_desc(gtp_ctx c, const gtp_events* ev) {
  if (!ev || ev->n_events < 0 || ev->t_end_ps <= 0) return fail(c, GTP_ERR_INVALID_ARG, "bad event descriptor");
  if (!ev->gate_off) return fail(c, GTP_ERR_INVALID_ARG, "null gate_off");
  if (ev->n_events > 0 && (!ev->t_ps || !ev->pin_bit || !ev->slew_ps))
    return fail(c, GTP_ERR_INVALID_ARG, "null event array");
  if (((uintptr_t)ev->t_ps | (uintptr_t)ev->pin_bit | (uintptr_t)ev->slew_ps) & 15)
    return fail(c, GTP_ERR_INVALID_ARG, "event arrays must be 16-byte aligned");
  if (c->n_gates == 0 && ev->n_events > 0) return fail(c, GTP_ERR_INVALID_ARG, "events without gates");
  int64_t ends[2] = {0, 0};
  HIPCHK(c, hipMemcpyAsync(&ends[0], ev->gate_off, 8, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(&ends[1], ev->gate_off + c->n_gates, 8, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (ends[0] != 0 || ends[1] != ev->n_events)
    return fail(c, GTP_ERR_INVALID_ARG, "gate_off must start at 0 and end at n_events (%lld, %lld)",
                (long long)ends[0], (long long)ends[1]);
  return GTP_OK;
}
}  // namespace

extern "C" {

gtp_status gtp_load_netlist(gtp_ctx c, int64_t n_gates, int64_t n_nets, const int32_t* gate_cell,
                            const int32_t* gate_out_net, const uint32_t* gate_init_bits) {
  TRY(need(c, true, false, false, false));
  HIPCHK(c, hipSetDevice(c->dev));
  if (n_gates < 0 || n_nets < 0 || n_gates >= (int64_t)INT32_MAX || n_nets >= (int64_t)INT32_MAX)
    return fail(c, GTP_ERR_INVALID_ARG, "n_gates=%lld n_nets=%lld", (long long)n_gates, (long long)n_nets);
  if (n_gates > 0 && (!gate_cell || !gate_out_net || !gate_init_bits))
    return fail(c, GTP_ERR_INVALID_ARG, "null netlist array");
  // from here on the old netlist is being replaced: until the new one is
  // checked and committed, the ctx holds none (a failed load leaves the
  // netlist, the events and every layout unloaded)
  c->net_ok = false;
  c->ev_ok = false;
  drop_pack(c);
  drop_batch(c);
  c->n_gates = 0;
  c->n_nets = 0;
  c->h_gate_cell.clear();
  TRY(ensure(c, c->gate_cell, (size_t)n_gates * 4));
  TRY(ensure(c, c->gate_out, (size_t)n_gates * 4));
  TRY(ensure(c, c->gate_init, (size_t)n_gates * 4));
  if (n_gates > 0) {
    HIPCHK(c, hipMemcpyAsync(c->gate_cell.p, gate_cell, (size_t)n_gates * 4, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->gate_out.p, gate_out_net, (size_t)n_gates * 4, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->gate_init.p, gate_init_bits, (size_t)n_gates * 4, hipMemcpyDeviceToDevice,
                             c->stream));
    TRY(ensure(c, c->first_bad, 256));
    TRY(fill_u64(c, c->first_bad.p, 1, 0ull));
    LAUNCH(c, "k_check_netlist", k_check_netlist, dim3(grid_for(n_gates, 256)), dim3(256), 0, ptr<int32_t>(c->gate_cell), ptr<int32_t>(c->gate_out), n_gates, c->n_cells, n_nets, ptr<int32_t>(c->first_bad));
    int32_t bad = 0;
    HIPCHK(c, hipMemcpyAsync(&bad, c->first_bad.p, 4, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (bad) return fail(c, GTP_ERR_INVALID_ARG, "a gate names a cell or output net out of range");
  }
  c->h_gate_cell.resize((size_t)n_gates);
  if (n_gates > 0)
    HIPCHK(c, hipMemcpy(c->h_gate_cell.data(), c->gate_cell.p, (size_t)n_gates * 4, hipMemcpyDeviceToHost));
  {
    // at most one driving gate per net: the adjoint then stores each gate's
    // load gradient into its net instead of adding it atomically
    std::vector<int32_t> out((size_t)n_gates);
    if (n_gates > 0) HIPCHK(c, hipMemcpy(out.data(), c->gate_out.p, (size_t)n_gates * 4, hipMemcpyDeviceToHost));
    std::vector<uint8_t> seen((size_t)std::max<int64_t>(n_nets, 1), 0);
    c->unique_out = true;
    for (int32_t o : out) {
      if (seen[(size_t)o]) {
        c->unique_out = false;
        break;
      }
      seen[(size_t)o] = 1;
    }
  }
  {
    double r = 0.0;
    for (int32_t cc : c->h_gate_cell) r += c->h_leak_max[(size_t)cc];
    c->r_bound = (double)GTP_MAX_LEAK_SCALE * r * 1e-6;
  }
  c->n_gates = n_gates;
  c->n_nets = n_nets;
  c->net_ok = true;
  c->ev_ok = false;
  drop_pack(c);
  drop_batch(c);
  return GTP_OK;
}

gtp_status gtp_load_events(gtp_ctx c, const gtp_events* ev, int validate) {
  TRY(need(c, true, true, false, false));
  HIPCHK(c, hipSetDevice(c->dev));
  c->bad_event = -1;
  TRY(check_event_desc(c, ev));
  c->ev = *ev;
  c->ev_ok = false;
  drop_pack(c);
  TRY(build_block_plan(c));
  c->ev_ok = true;
  if (c->par_ok) c->bins = bins_for(c, ev->t_end_ps);  // bins depend on t_end
  if (validate) {
    const gtp_status st = validate_events(c, *ev, c->plan_blk, c->n_blocks);
    if (st != GTP_OK) {
      c->ev_ok = false;
      return st;
    }
  }
  return GTP_OK;
}

gtp_status gtp_set_params(gtp_ctx c, const gtp_params* p) {
  TRY(need(c, true, false, false, false));
  if (!p || !(p->vdd > 0.0) || !std::isfinite(p->vdd) || p->bin_ps < 1 || p->bin_ps > (1 << 22) ||
      (p->sw_mode != 0 && p->sw_mode != 1) || p->glitch_clk_ps < 0)
    return fail(c, GTP_ERR_INVALID_ARG, "bad parameters");
  c->par = *p;
  BinSpec& B = c->bins;
  B.D = p->bin_ps;
  B.div = make_div32((uint32_t)B.D);
  B.r_bits = ceil_log2((uint64_t)B.D);
  B.tile_log2 = 8;
  B = bins_for(c, c->ev_ok ? c->ev.t_end_ps : 1);
  c->par_ok = true;
  drop_pack(c);
  drop_batch_packs(c);
  return GTP_OK;
}

gtp_status gtp_num_bins(gtp_ctx c, int64_t* n) {
  TRY(need(c, false, false, true, true));
  if (!n) return GTP_ERR_INVALID_ARG;
  *n = c->bins.n_bins;
  return GTP_OK;
}

gtp_status gtp_set_tuning(gtp_ctx c, const gtp_tuning* t) {
  if (!c || !t) return GTP_ERR_INVALID_ARG;
  if (t->algo < 0 || t->algo > 1) return fail(c, GTP_ERR_INVALID_ARG, "algo %d", t->algo);
  if (t->bins_per_tile_log2 != 0 && (t->bins_per_tile_log2 < 2 || t->bins_per_tile_log2 > 13))
    return fail(c, GTP_ERR_INVALID_ARG, "bins_per_tile_log2 %d", t->bins_per_tile_log2);
  if (t->tile_threads != 0 && t->tile_threads != 256 && t->tile_threads != 512 && t->tile_threads != 1024)
    return fail(c, GTP_ERR_INVALID_ARG, "tile_threads %d (0, 256, 512 or 1024)", t->tile_threads);
  if (t->unit_events < 0 || t->unit_events > kLaneEvents)
    return fail(c, GTP_ERR_INVALID_ARG, "unit_events %d (0..%d)", t->unit_events, kLaneEvents);
  if (t->gate_block_log2 != 0 && (t->gate_block_log2 < 6 || t->gate_block_log2 > 20))
    return fail(c, GTP_ERR_INVALID_ARG, "gate_block_log2 %d (0 or 6..20)", t->gate_block_log2);
  if (t->bins_per_tile_log2 != c->tun.bins_per_tile_log2 || t->unit_events != c->tun.unit_events ||
      t->gate_block_log2 != c->tun.gate_block_log2) {
    drop_pack(c);
    drop_batch_packs(c);
  }
  if (t->tile_threads != c->tun.tile_threads) drop_graph(c);
  c->tun = *t;
  return GTP_OK;
}

gtp_status gtp_get_tuning(gtp_ctx c, gtp_tuning* t) {
  if (!c || !t) return GTP_ERR_INVALID_ARG;
  *t = c->tun;
  if (c->pack_ok && t->bins_per_tile_log2 == 0) t->bins_per_tile_log2 = c->bins.tile_log2;
  if (t->tile_threads == 0) t->tile_threads = kTileThreads;
  if (t->unit_events == 0) t->unit_events = kDefaultUnitEvents;
  if (t->gate_block_log2 == 0) t->gate_block_log2 = kGateBlockLog2;
  return GTP_OK;
}

gtp_status gtp_plan_info(gtp_ctx c, gtp_plan_stats* out) {
  TRY(need(c, true, true, true, true));
  if (!out) return GTP_ERR_INVALID_ARG;
  HIPCHK(c, hipSetDevice(c->dev));
  TRY(build_pack(c));
  out->n_events_packed = c->pk.n_events;
  out->n_units = c->pk.n_units;
  out->n_groups = c->pk.n_groups;
  out->n_tiles = c->bins.n_tiles;
  out->tile_log2 = c->bins.tile_log2;
  out->max_tile_groups = c->pk.max_tile_groups;
  out->packed_bytes = c->pk.bytes;
  out->pack_ms = c->pack_ms;
  out->lane_steps = c->pk.lane_steps;
  return GTP_OK;
}

}  // extern "C"

namespace {
gtp_status final_bins(gtp_ctx c, float* power_mw, int32_t m) {
  const int64_t NB = c->bins.n_bins;
  TRY(scan_exclusive<int64_t, OpAdd>(c, ptr<int64_t>(c->S), ptr<int64_t>(c->exS), NB, (int64_t)0, OpAdd()));
  FinArgs f;
  f.X = ptr<int64_t>(c->X);
  f.S = ptr<int64_t>(c->S);
  f.exS = ptr<int64_t>(c->exS);
  f.L0 = ptr<unsigned long long>(c->L0);
  f.P = power_mw;
  f.n_bins = NB;
  f.D = c->bins.D;
  f.t_end = c->bins.t_end;
  f.out_scale = std::ldexp(1.0, -m) / (double)c->bins.D;
  LAUNCH(c, "k_finalize", k_finalize, dim3(grid_for(NB, 256)), dim3(256), 0, f);
  return GTP_OK;
}

// Per-call gate records in the pack's gate order, and the per-block partial
// sums of the initial leakage rates (l0_part).
// Per-call buffers of one packed forward (device pointers): gate records,
// initial-rate partials, the bins' X and in-tile step prefix, tile totals and
// rates at tile starts.
struct FwdScratch {
  GateParam* gparam;    // [n_gates]
  long long* l0_part;   // [l0_parts]
  int64_t* X;           // [n_bins]
  int64_t* S;           // [n_bins]
  long long* tile_tot;  // [n_tiles]
  long long* tile_base; // [n_tiles]
};

gtp_status gate_params_into(gtp_ctx c, const PackOut& pk, const float* net_load, const float* leak_scale,
                            GateParam* out, long long* l0_part) {
  if (c->n_gates == 0) return fill_u64(c, l0_part, 1, 0ull);
  const LibView L = lib_view(c);
  GateParamArgs a;
  a.gperm = pk.gperm;
  a.gcell = pk.gcell;
  a.gout = pk.gout;
  a.ginit = pk.ginit;
  a.net_load = net_load;
  a.leak_scale = leak_scale;
  a.meta = L.meta;
  a.leak = L.leak;
  a.wide = L.wide;
  a.n_gates = c->n_gates;
  a.rate_scale = rate_scale_of(pk.mfix);
  a.max_scale = GTP_MAX_LEAK_SCALE;
  a.load_cap = (float)c->load_cap;
  a.all_pins = c->all_pins;
  a.out = out;
  a.l0_part = l0_part;
  a.flag = ptr<int32_t>(c->flag);
  LAUNCH(c, "k_gate_params", k_gate_params, dim3(grid_for(c->n_gates, 256)), dim3(256), 0, a);
  return GTP_OK;
}

gtp_status gate_params_for(gtp_ctx c, const PackOut& pk, const float* net_load, const float* leak_scale) {
  TRY(ensure(c, c->gparam, (size_t)std::max<int64_t>(c->n_gates, 1) * sizeof(GateParam)));
  const int64_t nb = std::max<int64_t>(grid_for(c->n_gates, 256), 1);
  TRY(ensure(c, c->l0_part, (size_t)nb * 8));
  return gate_params_into(c, pk, net_load, leak_scale, ptr<GateParam>(c->gparam), ptr<long long>(c->l0_part));
}

int64_t l0_parts(gtp_ctx c) { return std::max<int64_t>(grid_for(c->n_gates, 256), 1); }

// L0 (the initial leakage rate) as one value, from the gate records' partials.
gtp_status sum_l0(gtp_ctx c) {
  TRY(ensure(c, c->L0, 8));
  LAUNCH(c, "k_sum_parts", k_sum_parts, dim3(1), dim3(1024), 0, (const long long*)ptr<long long>(c->l0_part),
         l0_parts(c), ptr<unsigned long long>(c->L0));
  return GTP_OK;
}

gtp_status gate_params(gtp_ctx c, const float* net_load, const float* leak_scale) {
  return gate_params_for(c, c->pk, net_load, leak_scale);
}

// Fields of the packed forward shared by every trace.
PackedFwdArgs packed_common(gtp_ctx c, int32_t m) {
  PackedFwdArgs a{};
  a.gparam = ptr<GateParam>(c->gparam);
  a.lib = lib_view(c);
  a.lut = lut_args(c, m);
  a.sw_mode = c->par.sw_mode;
  a.v2 = c->par.vdd * c->par.vdd;
  return a;
}

int tile_threads(gtp_ctx c) { return c->tun.tile_threads ? c->tun.tile_threads : kTileThreads; }

// Packed forward of one trace into X/S.
gtp_status packed_forward_for(gtp_ctx c, const PackOut& pk, const BinSpec& B, int64_t* X, int64_t* S,
                              long long* tile_tot = nullptr, const GateParam* gparam = nullptr) {
  PackedFwdArgs a = packed_common(c, pk.mfix);
  if (gparam) a.gparam = gparam;
  a.tile_tot = tile_tot;
  a.ev = pk.ev;
  a.desc = pk.desc;
  a.grp_off = pk.grp_off;
  a.tile_grp = pk.tile_grp;
  a.bins = B;
  a.X = X;
  a.S = S;
  const bool ph = pk.phases && pk.slot_quads > 0;
  a.phases = ph ? pk.phases : nullptr;
  a.ph_off = ph ? pk.ph_off : nullptr;
  a.slot_quads = ph ? pk.slot_quads : 0;
  const size_t lds = packed_lds_bytes(c, B.tile_log2) + (ph ? slot_bytes(pk.slot_quads) : 0);
  const int sl = slots_of(c);
  const int th = threads_for_slots(tile_threads(c), sl);
  const dim3 grid((unsigned)std::min<int64_t>(B.n_tiles, kMaxFwdGrid));
  // every quad from the LDS slots when every phase holds all its groups' quads
  const bool so = ph && pk.phases_full;
  a.rgl = pk.rgl;
  const bool gl = pk.rgl != nullptr;
#define GTP_PACKED_CASE(TH, SL)                                                                     \
  if (th == TH && sl == SL) {                                                                       \
    if (so && gl)                                                                                   \
      LAUNCH(c, "k_fwd_packed", (k_fwd_packed<TH, SL, true, true>), grid, dim3(TH), lds, a);        \
    else if (so)                                                                                    \
      LAUNCH(c, "k_fwd_packed", (k_fwd_packed<TH, SL, true, false>), grid, dim3(TH), lds, a);       \
    else if (gl)                                                                                    \
      LAUNCH(c, "k_fwd_packed", (k_fwd_packed<TH, SL, false, true>), grid, dim3(TH), lds, a);       \
    else                                                                                            \
      LAUNCH(c, "k_fwd_packed", (k_fwd_packed<TH, SL, false, false>), grid, dim3(TH), lds, a);      \
    return GTP_OK;                                                                                  \
  }
  GTP_PACKED_CASE(256, 8)
  GTP_PACKED_CASE(512, 8)
  GTP_PACKED_CASE(1024, 8)
  GTP_PACKED_CASE(256, 16)
  GTP_PACKED_CASE(512, 16)
#undef GTP_PACKED_CASE
  return fail(c, GTP_ERR_INVALID_ARG, "tile_threads %d", th);
}

// The whole packed forward of one trace (gate records already computed):
// the tile kernel leaves X, the within-tile prefix of the steps and the tile
// totals; one small kernel turns the totals into the rate at every tile
// start, one more gives the power.
gtp_status packed_power_into(gtp_ctx c, const PackOut& pk, const BinSpec& B, float* power_mw, const FwdScratch& w) {
  const int64_t NB = B.n_bins;
  TRY(packed_forward_for(c, pk, B, w.X, w.S, w.tile_tot, w.gparam));
  LAUNCH(c, "k_tile_base", k_tile_base, dim3(1), dim3(1024), 0, (const long long*)w.l0_part, l0_parts(c),
         (const long long*)w.tile_tot, (int64_t)B.n_tiles, w.tile_base);
  if (NB == 0) return GTP_OK;
  FinTileArgs f;
  f.X = w.X;
  f.exS = w.S;
  f.base = w.tile_base;
  f.tot = w.tile_tot;
  f.P = power_mw;
  f.n_bins = NB;
  f.D = B.D;
  f.t_end = B.t_end;
  f.tile_log2 = B.tile_log2;
  f.out_scale = std::ldexp(1.0, -pk.mfix) / (double)B.D;
  LAUNCH(c, "k_finalize_tiles", k_finalize_tiles, dim3(grid_for(NB, 256)), dim3(256), 0, f);
  return GTP_OK;
}

gtp_status packed_power(gtp_ctx c, const PackOut& pk, const BinSpec& B, float* power_mw) {
  const int64_t NB = B.n_bins;
  TRY(ensure(c, c->X, (size_t)std::max<int64_t>(NB, 1) * 8));
  TRY(ensure(c, c->S, (size_t)std::max<int64_t>(NB, 1) * 8));
  TRY(ensure(c, c->tile_tot, (size_t)std::max(B.n_tiles, 1) * 8));
  TRY(ensure(c, c->tile_base, (size_t)std::max(B.n_tiles, 1) * 8));
  const FwdScratch w{ptr<GateParam>(c->gparam), ptr<long long>(c->l0_part), ptr<int64_t>(c->X),
                     ptr<int64_t>(c->S),        ptr<long long>(c->tile_tot), ptr<long long>(c->tile_base)};
  return packed_power_into(c, pk, B, power_mw, w);
}

// ---------------------------------------------------------------------------
// batched traces
// ---------------------------------------------------------------------------
void drop_graph(gtp_ctx c) {
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  c->gexec = nullptr;
  c->graph = nullptr;
  c->gkey[0] = c->gkey[1] = c->gkey[2] = nullptr;
}

void drop_batch_packs(gtp_ctx c) {
  drop_graph(c);
  if (c->batch_packed) (void)hipStreamSynchronize(c->stream);
  for (auto& t : c->batch) {
    if (t.pk.ev || t.pk.gperm) {
      c->dev_bytes -= t.pk.bytes;
      pack_free(&t.pk);
    }
  }
  c->batch_packed = false;
}

void drop_batch(gtp_ctx c) {
  drop_batch_packs(c);
  for (auto& t : c->batch) release(c, t.plan);
  c->batch.clear();
  c->batch_total_bins = 0;
  c->batch_items = 0;
}

// Packs every trace with one bin-per-tile choice, builds the trace table, the
// work items (largest first) and the finalize table.
gtp_status build_batch(gtp_ctx c) {
  if (c->batch_packed) return GTP_OK;
  drop_batch_packs(c);
  const int32_t nt = (int32_t)c->batch.size();
  // one tile size for all traces (the queue balances uneven traces)
  const BinSpec B0 = c->bins;
  const int lb = c->tun.bins_per_tile_log2 ? c->tun.bins_per_tile_log2
                                           : std::min(12, std::max(2, kTimeBits - B0.r_bits));
  if (packed_lds_bytes(c, lb) + kBatchStaticLds > kMaxLds)
    return fail(c, GTP_ERR_UNSUPPORTED, "tile of 2^%d bins and the library image exceed the LDS", lb);
  // the traces share one set of gate records, so one gate order: by events
  // over all traces
  std::vector<int64_t> wt((size_t)c->n_gates, 0);
  if (c->n_gates > 0) {
    std::vector<int64_t> go((size_t)c->n_gates + 1);
    for (int32_t i = 0; i < nt; ++i) {
      HIPCHK(c, hipMemcpy(go.data(), c->batch[i].ev.gate_off, go.size() * 8, hipMemcpyDeviceToHost));
      for (int64_t g = 0; g < c->n_gates; ++g) wt[g] += go[g + 1] - go[g];
    }
  }
  gtp_tuning saved = c->tun;
  c->tun.bins_per_tile_log2 = lb;
  std::vector<TraceDev> tab((size_t)nt);
  std::vector<FinTrace> fin((size_t)nt);
  std::vector<std::pair<int64_t, int2>> items;
  int64_t off = 0, toff = 0, boff = 0;
  for (int32_t i = 0; i < nt; ++i) {
    auto& t = c->batch[i];
    t.bins = bins_for(c, t.ev.t_end_ps);
    const gtp_status st = pack_for(c, t.ev, t.plan, t.bins, t.pk, t.pack_ms, nullptr, nullptr, &wt);
    if (st != GTP_OK) {
      c->tun = saved;
      return st;
    }
    t.bin_off = off;
    const bool ph = t.pk.phases && t.pk.slot_quads > 0;
    tab[i] = TraceDev{t.pk.ev,
                      t.pk.rgl,
                      ph ? t.pk.phases : nullptr,
                      ph ? t.pk.ph_off : nullptr,
                      ph ? t.pk.slot_quads : 0,
                      t.pk.desc,
                      t.pk.grp_off,
                      t.pk.tile_grp,
                      t.bins,
                      off,
                      toff};
    fin[i] = FinTrace{off, t.bins.n_bins, t.bins.t_end, toff, t.bins.n_tiles, boff};
    boff += (t.bins.n_bins + kFinBins - 1) / kFinBins;
    off += t.bins.n_bins;
    toff += t.bins.n_tiles;
    // events per tile, for the largest-first order
    const int32_t ntile = t.bins.n_tiles;
    std::vector<int32_t> tg((size_t)ntile + 1);
    HIPCHK(c, hipMemcpy(tg.data(), t.pk.tile_grp, (size_t)(ntile + 1) * 4, hipMemcpyDeviceToHost));
    std::vector<int64_t> go((size_t)t.pk.n_groups + 1);
    HIPCHK(c, hipMemcpy(go.data(), t.pk.grp_off, (size_t)(t.pk.n_groups + 1) * 8, hipMemcpyDeviceToHost));
    for (int32_t k = 0; k < ntile; ++k) items.push_back({go[tg[k + 1]] - go[tg[k]], make_int2(i, k)});
  }
  c->tun = saved;
  // one fixed-point exponent for the batch (the traces share the gate
  // records): the smallest any trace needs
  {
    int32_t m = kMaxMfix;
    for (auto& t : c->batch) m = std::min(m, t.pk.mfix);
    for (auto& t : c->batch) t.pk.mfix = m;
  }
  std::stable_sort(items.begin(), items.end(),
                   [](const std::pair<int64_t, int2>& x, const std::pair<int64_t, int2>& y) { return x.first > y.first; });
  std::vector<int2> it(items.size());
  for (size_t j = 0; j < items.size(); ++j) it[j] = items[j].second;
  c->batch_total_bins = off;
  c->batch_total_tiles = toff;
  c->batch_fin_blocks = boff;
  c->batch_items = (int64_t)it.size();
  TRY(ensure(c, c->b_tab, tab.size() * sizeof(TraceDev)));
  TRY(ensure(c, c->b_fin, fin.size() * sizeof(FinTrace)));
  TRY(ensure(c, c->b_items, std::max<size_t>(it.size(), 1) * sizeof(int2)));
  TRY(ensure(c, c->b_tile_tot, (size_t)std::max<int64_t>(toff, 1) * 8));
  TRY(ensure(c, c->b_tile_base, (size_t)std::max<int64_t>(toff, 1) * 8));
  if (nt > 0) {
    HIPCHK(c, hipMemcpy(c->b_tab.p, tab.data(), tab.size() * sizeof(TraceDev), hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->b_fin.p, fin.data(), fin.size() * sizeof(FinTrace), hipMemcpyHostToDevice));
  }
  if (!it.empty()) HIPCHK(c, hipMemcpy(c->b_items.p, it.data(), it.size() * sizeof(int2), hipMemcpyHostToDevice));
  const int64_t NB = std::max<int64_t>(off, 1);
  TRY(ensure(c, c->b_X, (size_t)NB * 8));
  TRY(ensure(c, c->b_S, (size_t)NB * 8));
  TRY(ensure(c, c->gparam, (size_t)std::max<int64_t>(c->n_gates, 1) * sizeof(GateParam)));
  TRY(ensure(c, c->L0, 8));
  TRY(ensure(c, c->l0_part, (size_t)l0_parts(c) * 8));
  c->batch_packed = true;
  return GTP_OK;
}

// Every launch of a batched forward (no allocation, no synchronisation: safe
// to record in a graph).
gtp_status batched_enqueue(gtp_ctx c, const float* net_load, const float* leak_scale, float* power_mw) {
  TRY(gate_params_for(c, c->batch[0].pk, net_load, leak_scale));
  TRY(sum_l0(c));
  const int lb = c->batch[0].bins.tile_log2;
  if (c->batch_items > 0) {
    BatchFwdArgs a;
    a.base = packed_common(c, c->batch[0].pk.mfix);
    a.traces = ptr<TraceDev>(c->b_tab);
    a.items = ptr<int2>(c->b_items);
    a.n_items = c->batch_items;
    a.X = ptr<int64_t>(c->b_X);
    a.S = ptr<int64_t>(c->b_S);
    a.tile_tot = ptr<long long>(c->b_tile_tot);
    int32_t sq = 0;  // every trace's pack has the same slot size (same tile size)
    bool so = true;  // every trace's phases hold all their groups' quads
    for (auto& t : c->batch) {
      if (t.pk.phases) sq = std::max(sq, t.pk.slot_quads);
      so = so && t.pk.phases && t.pk.slot_quads > 0 && t.pk.phases_full;
    }
    const size_t lds = packed_lds_bytes(c, lb) + slot_bytes(sq);
    const int sl = slots_of(c);
    const int th = threads_for_slots(tile_threads(c), sl);
    const dim3 grid((unsigned)c->batch_items);   // one workgroup per (trace, tile) item
    const bool gl = c->par.glitch_clk_ps > 0;
#define GTP_BATCH_CASE(TH, SL)                                                                       \
  if (th == TH && sl == SL) {                                                                        \
    if (so && gl)                                                                                    \
      LAUNCH(c, "k_fwd_batched", (k_fwd_batched<TH, SL, true, true>), grid, dim3(TH), lds, a);       \
    else if (so)                                                                                     \
      LAUNCH(c, "k_fwd_batched", (k_fwd_batched<TH, SL, true, false>), grid, dim3(TH), lds, a);      \
    else if (gl)                                                                                     \
      LAUNCH(c, "k_fwd_batched", (k_fwd_batched<TH, SL, false, true>), grid, dim3(TH), lds, a);      \
    else                                                                                             \
      LAUNCH(c, "k_fwd_batched", (k_fwd_batched<TH, SL, false, false>), grid, dim3(TH), lds, a);     \
  }
    GTP_BATCH_CASE(256, 8)
    GTP_BATCH_CASE(512, 8)
    GTP_BATCH_CASE(1024, 8)
    GTP_BATCH_CASE(256, 16)
    GTP_BATCH_CASE(512, 16)
#undef GTP_BATCH_CASE
  }
  const int64_t NB = c->batch_total_bins;
  const int32_t n_traces = (int32_t)c->batch.size();
  if (c->batch_total_tiles > 0)
    LAUNCH(c, "k_tile_base_batched", k_tile_base_batched, dim3((unsigned)n_traces), dim3(1024), 0,
           (const unsigned long long*)ptr<unsigned long long>(c->L0), (const FinTrace*)ptr<FinTrace>(c->b_fin),
           (const long long*)ptr<long long>(c->b_tile_tot), ptr<long long>(c->b_tile_base));
  FinBatchArgs f;
  f.X = ptr<int64_t>(c->b_X);
  f.S = ptr<int64_t>(c->b_S);
  f.base = ptr<long long>(c->b_tile_base);
  f.tot = ptr<long long>(c->b_tile_tot);
  f.traces = ptr<FinTrace>(c->b_fin);
  f.n_traces = n_traces;
  f.tile_log2 = lb;
  f.P = power_mw;
  f.total_bins = NB;
  f.D = c->bins.D;
  f.out_scale = std::ldexp(1.0, -c->batch[0].pk.mfix) / (double)c->bins.D;
  if (NB > 0)
    LAUNCH(c, "k_finalize_batched", k_finalize_batched, dim3((unsigned)c->batch_fin_blocks), dim3(kFinBins), 0, f);
  return GTP_OK;
}

// Records batched_enqueue into a graph on a private capture stream.
gtp_status capture_batched(gtp_ctx c, const float* net_load, const float* leak_scale, float* power_mw) {
  drop_graph(c);
  if (!c->cap_stream) HIPCHK(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
  hipStream_t saved = c->stream;
  const bool prof = c->prof_on;
  c->prof_on = false;
  c->stream = c->cap_stream;
  hipError_t e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal);
  gtp_status st = GTP_OK;
  if (e == hipSuccess) st = batched_enqueue(c, net_load, leak_scale, power_mw);
  hipGraph_t g = nullptr;
  const hipError_t e2 = (e == hipSuccess) ? hipStreamEndCapture(c->cap_stream, &g) : e;
  c->stream = saved;
  c->prof_on = prof;
  if (e != hipSuccess || e2 != hipSuccess || st != GTP_OK) {
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    if (st != GTP_OK) return st;
    return fail(c, GTP_ERR_HIP, "graph capture failed: %s", hipGetErrorString(e != hipSuccess ? e : e2));
  }
  c->graph = g;
  HIPCHK(c, hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0));
  c->gkey[0] = net_load;
  c->gkey[1] = leak_scale;
  c->gkey[2] = power_mw;
  return GTP_OK;
}
}  // namespace

extern "C" {

gtp_status gtp_forward(gtp_ctx c, const float* net_load_ff, const float* leak_scale, float* power_mw) {
  TRY(need(c, true, true, true, true));
  if (!net_load_ff || !power_mw) return fail(c, GTP_ERR_INVALID_ARG, "null forward argument");
  HIPCHK(c, hipSetDevice(c->dev));
  const int64_t NB = c->bins.n_bins;
  TRY(ensure(c, c->X, (size_t)NB * 8));
  TRY(ensure(c, c->S, (size_t)NB * 8));
  TRY(ensure(c, c->exS, (size_t)NB * 8));
  const int64_t N = c->ev.n_events;
  // the packed layout also fixes the fixed-point exponent of this event set,
  // which the one-gate-per-thread path uses too (so both give the same bits)
  TRY(build_pack(c));
  const int32_t m = c->pk.mfix;
  if (c->tun.algo == 0) {
    TRY(gate_params(c, net_load_ff, leak_scale));
    return packed_power(c, c->pk, c->bins, power_mw);
  } else {
    TRY(gate_prep(c, net_load_ff, leak_scale, m));
    TRY(fill_u64(c, c->X.p, NB, 0ull));
    TRY(fill_u64(c, c->S.p, NB, 0ull));
    if (c->n_gates > 0 && N > 0) {
      SerialArgs a;
      a.ev = ev_view(c);
      a.gprep = ptr<GatePrep>(c->gprep);
      a.lib = lib_view(c);
      a.lut = lut_args(c, m);
      a.bins = c->bins;
      a.glitch_clk = c->par.glitch_clk_ps;
      a.X = ptr<unsigned long long>(c->X);
      a.S = ptr<unsigned long long>(c->S);
      LAUNCH(c, "k_gate_serial", k_gate_serial, dim3(grid_for(c->n_gates, kFwdThreads)), dim3(kFwdThreads), lib_lds_bytes(c), a);
    }
  }
  return final_bins(c, power_mw, m);
}

gtp_status gtp_forward_noalloc(gtp_ctx c, const float* net_load_ff, const float* leak_scale, float* power_mw) {
  TRY(need(c, true, true, true, true));
  if (!net_load_ff || !power_mw) return fail(c, GTP_ERR_INVALID_ARG, "null forward argument");
  if (c->tun.algo != 0) return fail(c, GTP_ERR_UNSUPPORTED, "the allocation-free forward runs the packed path (algo 0)");
  if (!c->pack_ok)
    return fail(c, GTP_ERR_NOT_LOADED,
                "the packed layout is not built: call gtp_plan_info or gtp_forward once after loading the events");
  if (!c->scratch_dev) return fail(c, GTP_ERR_HIP, "no scratch address for device %d", c->dev);
  HIPCHK(c, hipSetDevice(c->dev));
  const BinSpec& B = c->bins;
  // carve the per-call buffers from the scratch array (256-byte aligned)
  auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const size_t s_gp = up((size_t)std::max<int64_t>(c->n_gates, 1) * sizeof(GateParam));
  const size_t s_l0 = up((size_t)l0_parts(c) * 8);
  const size_t s_bin = up((size_t)std::max<int64_t>(B.n_bins, 1) * 8);
  const size_t s_tile = up((size_t)std::max(B.n_tiles, 1) * 8);
  const size_t need_bytes = s_gp + s_l0 + 2 * s_bin + 2 * s_tile;
  if (need_bytes > kScratchBytes)
    return fail(c, GTP_ERR_UNSUPPORTED,
                "%lld gates and %lld bins need %zu bytes of scratch; the allocation-free forward holds %zu",
                (long long)c->n_gates, (long long)B.n_bins, need_bytes, kScratchBytes);
  unsigned char* base = static_cast<unsigned char*>(c->scratch_dev);
  FwdScratch w;
  w.gparam = reinterpret_cast<GateParam*>(base);
  w.l0_part = reinterpret_cast<long long*>(base + s_gp);
  w.X = reinterpret_cast<int64_t*>(base + s_gp + s_l0);
  w.S = reinterpret_cast<int64_t*>(base + s_gp + s_l0 + s_bin);
  w.tile_tot = reinterpret_cast<long long*>(base + s_gp + s_l0 + 2 * s_bin);
  w.tile_base = reinterpret_cast<long long*>(base + s_gp + s_l0 + 2 * s_bin + s_tile);
  // no profiling events here (creating one is a driver allocation)
  const bool prof = c->prof_on;
  c->prof_on = false;
  gtp_status st = gate_params_into(c, c->pk, net_load_ff, leak_scale, w.gparam, w.l0_part);
  if (st == GTP_OK) st = packed_power_into(c, c->pk, B, power_mw, w);
  c->prof_on = prof;
  return st;
}

gtp_status gtp_load_traces(gtp_ctx c, int32_t n_traces, const gtp_events* traces, int validate) {
  TRY(need(c, true, true, false, true));
  HIPCHK(c, hipSetDevice(c->dev));
  c->bad_event = -1;
  if (n_traces < 1 || !traces) return fail(c, GTP_ERR_INVALID_ARG, "need at least one trace");
  drop_batch(c);
  c->batch.resize((size_t)n_traces);
  for (int32_t i = 0; i < n_traces; ++i) {
    auto& t = c->batch[i];
    gtp_status st = check_event_desc(c, &traces[i]);
    if (st == GTP_OK) {
      t.ev = traces[i];
      st = block_plan_for(c, t.ev, t.plan, t.n_blocks);
    }
    if (st == GTP_OK && validate) st = validate_events(c, t.ev, t.plan, t.n_blocks);
    if (st != GTP_OK) {
      const std::string m = c->err;
      drop_batch(c);
      return fail(c, st, "trace %d: %s", (int)i, m.c_str());
    }
  }
  return GTP_OK;
}

gtp_status gtp_batch_bins(gtp_ctx c, int64_t* total, int64_t* offsets) {
  TRY(need(c, true, true, false, true));
  if (c->batch.empty()) return fail(c, GTP_ERR_NOT_LOADED, "no batch loaded");
  if (!total) return GTP_ERR_INVALID_ARG;
  int64_t off = 0;
  for (size_t i = 0; i < c->batch.size(); ++i) {
    if (offsets) offsets[i] = off;
    off += bins_for(c, c->batch[i].ev.t_end_ps).n_bins;
  }
  if (offsets) offsets[c->batch.size()] = off;
  *total = off;
  return GTP_OK;
}

gtp_status gtp_forward_batched(gtp_ctx c, const float* net_load_ff, const float* leak_scale, float* power_mw,
                               int use_graph) {
  TRY(need(c, true, true, false, true));
  if (c->batch.empty()) return fail(c, GTP_ERR_NOT_LOADED, "no batch loaded");
  if (!net_load_ff || !power_mw) return fail(c, GTP_ERR_INVALID_ARG, "null forward argument");
  HIPCHK(c, hipSetDevice(c->dev));
  TRY(build_batch(c));
  if (!use_graph) return batched_enqueue(c, net_load_ff, leak_scale, power_mw);
  if (!c->gexec || c->gkey[0] != net_load_ff || c->gkey[1] != leak_scale || c->gkey[2] != power_mw)
    TRY(capture_batched(c, net_load_ff, leak_scale, power_mw));
  prof_begin(c, "graph_forward_batched");
  HIPCHK(c, hipGraphLaunch(c->gexec, c->stream));
  prof_end(c);
  return GTP_OK;
}

gtp_status gtp_forward_trace(gtp_ctx c, int32_t trace, const float* net_load_ff, const float* leak_scale,
                             float* power_mw) {
  TRY(need(c, true, true, false, true));
  if (trace < 0 || trace >= (int32_t)c->batch.size()) return fail(c, GTP_ERR_INVALID_ARG, "trace %d", (int)trace);
  if (!net_load_ff || !power_mw) return fail(c, GTP_ERR_INVALID_ARG, "null forward argument");
  HIPCHK(c, hipSetDevice(c->dev));
  TRY(build_batch(c));
  const auto& t = c->batch[trace];
  const int64_t NB = t.bins.n_bins;
  TRY(ensure(c, c->X, (size_t)NB * 8));
  TRY(ensure(c, c->S, (size_t)NB * 8));
  TRY(ensure(c, c->exS, (size_t)NB * 8));
  TRY(gate_params_for(c, t.pk, net_load_ff, leak_scale));
  return packed_power(c, t.pk, t.bins, power_mw);
}

}  // extern "C"

namespace {
// Signature of the loaded workload for the autotune cache.
std::string tune_key(gtp_ctx c) {
  hipDeviceProp_t pr;
  std::string dev = "gpu";
  if (hipGetDeviceProperties(&pr, c->dev) == hipSuccess) dev = pr.gcnArchName;
  (void)hipGetLastError();
  int64_t nev = 0, nb = 0;
  if (!c->batch.empty()) {
    for (auto& t : c->batch) {
      nev += t.ev.n_events;
      nb += bins_for(c, t.ev.t_end_ps).n_bins;
    }
  } else {
    nev = c->ev.n_events;
    nb = c->bins.n_bins;
  }
  std::ostringstream k;
  k << dev << "/cu" << c->n_cu << "/g" << c->n_gates << "/c" << c->n_cells << "/e" << nev << "/b" << nb << "/d"
    << c->bins.D << "/t" << c->batch.size();
  return k.str();
}

bool tune_cache_lookup(const char* path, const std::string& key, gtp_tuning* t) {
  if (!path) return false;
  std::ifstream f(path);
  std::string line;
  const std::string pat = "\"key\": \"" + key + "\"";
  while (std::getline(f, line)) {
    if (line.find(pat) == std::string::npos) continue;
    gtp_tuning r{0, 0, 0, 0, 0};
    auto field = [&](const char* name, int32_t* v) {
      const std::string n = std::string("\"") + name + "\": ";
      const size_t p = line.find(n);
      if (p == std::string::npos) return false;
      *v = (int32_t)std::strtol(line.c_str() + p + n.size(), nullptr, 10);
      return true;
    };
    if (field("algo", &r.algo) && field("bins_per_tile_log2", &r.bins_per_tile_log2) &&
        field("tile_threads", &r.tile_threads) && field("unit_events", &r.unit_events) &&
        field("gate_block_log2", &r.gate_block_log2)) {
      *t = r;
      return true;
    }
  }
  return false;
}

void tune_cache_append(const char* path, const std::string& key, const gtp_tuning& t, double ms) {
  if (!path) return;
  std::ofstream f(path, std::ios::app);
  f << "{\"key\": \"" << key << "\", \"algo\": " << t.algo << ", \"bins_per_tile_log2\": " << t.bins_per_tile_log2
    << ", \"tile_threads\": " << t.tile_threads << ", \"unit_events\": " << t.unit_events
    << ", \"gate_block_log2\": " << t.gate_block_log2 << ", \"ms\": " << ms << "}\n";
}
}  // namespace

extern "C" {

gtp_status gtp_autotune(gtp_ctx c, const char* cache_json_path) {
  TRY(need(c, true, true, false, true));
  const bool batched = !c->batch.empty();
  if (!batched && !c->ev_ok) return fail(c, GTP_ERR_NOT_LOADED, "no events or batch loaded");
  HIPCHK(c, hipSetDevice(c->dev));
  const std::string key = tune_key(c);
  gtp_tuning cached;
  if (tune_cache_lookup(cache_json_path, key, &cached)) return gtp_set_tuning(c, &cached);
  // inputs: unit loads, unit scales; output sized for the workload
  int64_t nb = c->bins.n_bins;
  if (batched) TRY(gtp_batch_bins(c, &nb, nullptr));
  TRY(ensure(c, c->tun_in, (size_t)(c->n_nets + 2) * 4));
  TRY(fill_u64(c, c->tun_in.p, (c->n_nets + 2) / 2, 0x3f8000003f800000ull));
  TRY(ensure(c, c->tun_out, (size_t)std::max<int64_t>(nb, 1) * 4));
  const float* load = ptr<float>(c->tun_in);
  float* out = ptr<float>(c->tun_out);
  auto run = [&]() -> gtp_status {
    if (batched) return gtp_forward_batched(c, load, nullptr, out, 0);
    return gtp_forward(c, load, nullptr, out);
  };
  const bool prof = c->prof_on;
  c->prof_on = false;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(c, hipEventCreate(&e0));
  HIPCHK(c, hipEventCreate(&e1));
  gtp_tuning best{0, 0, 0, 0, 0};
  double best_ms = 1e30;
  const int tiles[] = {11, 12, 13};
  const int threads[] = {512, 1024};
  const int units[] = {8, 16};
  const int gblocks[] = {12, 13};
  for (int tl : tiles)
    for (int un : units)
      for (int gbl : gblocks)
        for (int th : threads) {
          gtp_tuning t{0, tl, th, un, gbl};
          if (gtp_set_tuning(c, &t) != GTP_OK) continue;
          if (run() != GTP_OK || hipStreamSynchronize(c->stream) != hipSuccess) {  // builds the layout
            (void)hipGetLastError();
            continue;
          }
          const int reps = 3;
          (void)hipEventRecord(e0, c->stream);
          gtp_status st = GTP_OK;
          for (int r = 0; r < reps && st == GTP_OK; ++r) st = run();
          (void)hipEventRecord(e1, c->stream);
          (void)hipEventSynchronize(e1);
          float ms = 0.f;
          (void)hipEventElapsedTime(&ms, e0, e1);
          if (st == GTP_OK && ms / reps < best_ms) {
            best_ms = ms / reps;
            best = t;
          }
        }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  c->prof_on = prof;
  if (best_ms >= 1e30) return fail(c, GTP_ERR_UNSUPPORTED, "no candidate tuning ran");
  TRY(gtp_set_tuning(c, &best));
  tune_cache_append(cache_json_path, key, best, best_ms);
  return GTP_OK;
}

gtp_status gtp_adjoint(gtp_ctx c, const float* net_load_ff, const float* leak_scale, const float* grad_power,
                       float* grad_net_load, float* grad_leak_scale) {
  TRY(need(c, true, true, true, true));
  if (!net_load_ff || !grad_power || !grad_net_load || !grad_leak_scale)
    return fail(c, GTP_ERR_INVALID_ARG, "null adjoint argument");
  HIPCHK(c, hipSetDevice(c->dev));
  const int64_t NB = c->bins.n_bins;
  bool packed = c->tun.algo == 0;
  if (packed) {
    TRY(build_pack(c));
    TRY(build_pack_adj(c));
    TRY(adj_plan(c));
    packed = adj_lds_bytes(c, c->adj_max_gb) <= kMaxLds;  // else the gate-major kernel
  }
  TRY(ensure(c, c->adj_w, (size_t)NB * 8));
  TRY(ensure(c, c->adj_c, (size_t)NB * 8));
  TRY(ensure(c, c->adj_exc, (size_t)NB * 8));
  TRY(ensure(c, c->adj_wg, (size_t)NB * 16));
  TRY(ensure(c, c->adj_total, 8));
  TRY(ensure(c, c->gC, (size_t)std::max<int64_t>(std::max(c->n_nets, c->n_gates), 1) * 8));
  TRY(ensure(c, c->gL, (size_t)std::max<int64_t>(c->n_gates, 1) * 8));
  AdjBinArgs ab;
  ab.gP = grad_power;
  ab.c = ptr<double>(c->adj_c);
  ab.wgtmp = ptr<double>(c->adj_w);
  ab.n_bins = NB;
  ab.D = c->bins.D;
  ab.t_end = c->bins.t_end;
  LAUNCH(c, "k_adj_bins", k_adj_bins, dim3(grid_for(NB, 256)), dim3(256), 0, ab);
  TRY(scan_exclusive<double, OpAdd>(c, ptr<double>(c->adj_c), ptr<double>(c->adj_exc), NB, 0.0, OpAdd()));
  const double v2 = c->par.vdd * c->par.vdd;
  const float dsw_rise = (float)(c->par.sw_mode == 0 ? 0.5 * v2 : v2);
  const float dsw_fall = (float)(c->par.sw_mode == 0 ? 0.5 * v2 : 0.0);
  if (packed) {
    TRY(ensure(c, c->adj_gtile, (size_t)std::max(c->bins.n_tiles, 1) * 8));
    LAUNCH(c, "k_adj_suffix_tiles", k_adj_suffix_tiles, dim3(grid_for(NB, 256)), dim3(256), 0,
           (const double*)ptr<double>(c->adj_w), (const double*)ptr<double>(c->adj_c),
           (const double*)ptr<double>(c->adj_exc), ptr<float2>(c->adj_wg), ptr<double>(c->adj_gtile),
           ptr<double>(c->adj_total), NB, (int32_t)c->bins.tile_log2);
    TRY(gate_params(c, net_load_ff, leak_scale));
    if (c->adj_n_items > 0) {
      const PackOut& pk = adj_pack(c);
      AdjPackedArgs a;
      a.f = packed_common(c, pk.mfix);
      a.f.ev = pk.ev;
      a.f.desc = pk.desc;
      a.f.grp_off = pk.grp_off;
      a.f.tile_grp = pk.tile_grp;
      a.f.bins = c->bins;
      a.f.rgl = pk.rgl;
      a.entries = ptr<int4>(c->adj_entries);
      a.items = ptr<AdjItem>(c->adj_items);
      a.gb_start = ptr<int32_t>(c->adj_gbs);
      a.part = ptr<double2>(c->adj_part);
      a.last_w = (int32_t)(c->bins.t_end - (c->bins.n_bins - 1) * c->bins.D);
      a.wg = ptr<float2>(c->adj_wg);
      a.gtile = ptr<double>(c->adj_gtile);
      a.dsw_rise = dsw_rise;
      a.dsw_fall = dsw_fall;
      a.slot_quads = adj_slot_quads(c, c->adj_max_gb);
      const dim3 gi((unsigned)c->adj_n_items);
      const size_t al = adj_lds_bytes(c, c->adj_max_gb);
      const bool gl = pk.rgl != nullptr;
      const bool to = c->adj_tab_only;
#define ADJ_LAUNCH(TH, SL, GL, TO) LAUNCH(c, "k_adjoint_packed", (k_adjoint_packed<TH, SL, GL, TO>), gi, dim3(TH), al, a)
      if (slots_of(c) == 8) {
        if (gl) {
          if (to) ADJ_LAUNCH(1024, 8, true, true); else ADJ_LAUNCH(1024, 8, true, false);
        } else {
          if (to) ADJ_LAUNCH(1024, 8, false, true); else ADJ_LAUNCH(1024, 8, false, false);
        }
      } else {
        if (gl) {
          if (to) ADJ_LAUNCH(512, 16, true, true); else ADJ_LAUNCH(512, 16, true, false);
        } else {
          if (to) ADJ_LAUNCH(512, 16, false, true); else ADJ_LAUNCH(512, 16, false, false);
        }
      }
#undef ADJ_LAUNCH
    }
    if (c->n_nets > 0)
      LAUNCH(c, "k_fill_i32", k_fill_i32, dim3(grid_for(c->n_nets, 256)), dim3(256), 0, (int32_t*)grad_net_load,
             c->n_nets, 0);
    if (c->n_gates > 0) {
      AdjOutSortedArgs o;
      o.part = ptr<double2>(c->adj_part);
      o.gb_row = ptr<int64_t>(c->adj_gbrow);
      o.gb_rows = ptr<int32_t>(c->adj_gbrows);
      o.gb_start = ptr<int32_t>(c->adj_gbs);
      const PackOut& pa = adj_pack(c);   // the layout the adjoint's partial rows follow
      o.n_gb = pa.n_gb;
      o.total = ptr<double>(c->adj_total);
      o.gperm = pa.gperm;
      o.gcell = pa.gcell;
      o.gate_out = ptr<int32_t>(c->gate_out);
      o.gate_init = ptr<uint32_t>(c->gate_init);
      o.meta = lib_view(c).meta;
      o.leak = lib_view(c).leak;
      o.wide = lib_view(c).wide;
      o.grad_load = grad_net_load;
      o.grad_scale = grad_leak_scale;
      o.n_gates = c->n_gates;
      o.unique_out = c->unique_out ? 1 : 0;
      o.all_pins = c->all_pins;
      LAUNCH(c, "k_adj_out_sorted", k_adj_out_sorted, dim3(grid_for(c->n_gates, 256)), dim3(256), 0, o);
    }
    return GTP_OK;
  }
  LAUNCH(c, "k_adj_suffix", k_adj_suffix, dim3(grid_for(NB, 256)), dim3(256), 0, (const double*)ptr<double>(c->adj_w), (const double*)ptr<double>(c->adj_c), (const double*)ptr<double>(c->adj_exc), ptr<double2>(c->adj_wg), ptr<double>(c->adj_total), NB);
  TRY(gate_prep(c, net_load_ff, leak_scale, kAnyMfix));
  TRY(fill_u64(c, c->gC.p, c->n_nets, 0ull));
  TRY(fill_u64(c, c->gL.p, c->n_gates, 0ull));
  if (c->n_blocks > 0) {
    AdjArgs a;
    a.ev = ev_view(c);
    a.plan = ptr<uint2>(c->plan_blk);
    a.gprep = ptr<GatePrep>(c->gprep);
    a.gate_out = ptr<int32_t>(c->gate_out);
    a.lib = lib_view(c);
    a.lut = lut_args(c, kAnyMfix);
    a.bins = c->bins;
    a.wg = ptr<double2>(c->adj_wg);
    a.dsw_rise = dsw_rise;
    a.dsw_fall = dsw_fall;
    a.glitch_clk = c->par.glitch_clk_ps;
    a.gC = ptr<double>(c->gC);
    a.gL = ptr<double>(c->gL);
    LAUNCH(c, "k_adjoint_events", k_adjoint_events, dim3(grid_for(c->n_blocks, kFwdThreads)), dim3(kFwdThreads), lib_lds_bytes(c), a);
  }
  const int64_t n = std::max(c->n_nets, c->n_gates);
  if (n > 0) {
    AdjOutArgs o;
    o.gC = ptr<double>(c->gC);
    o.gL = ptr<double>(c->gL);
    o.total = ptr<double>(c->adj_total);
    o.gate_cell = ptr<int32_t>(c->gate_cell);
    o.gate_init = ptr<uint32_t>(c->gate_init);
    o.meta = lib_view(c).meta;
    o.leak = lib_view(c).leak;
    o.wide = lib_view(c).wide;
    o.grad_load = grad_net_load;
    o.grad_scale = grad_leak_scale;
    o.n_nets = c->n_nets;
    o.n_gates = c->n_gates;
    o.all_pins = c->all_pins;
    LAUNCH(c, "k_adj_out", k_adj_out, dim3(grid_for(n, 256)), dim3(256), 0, o);
  }
  return GTP_OK;
}

gtp_status gtp_gate_report(gtp_ctx c, const float* net_load_ff, const float* leak_scale, const float* power_mw,
                           double* gate_energy_fj, double* totals) {
  TRY(need(c, true, true, true, true));
  if (!net_load_ff || !gate_energy_fj || !totals) return fail(c, GTP_ERR_INVALID_ARG, "null report argument");
  HIPCHK(c, hipSetDevice(c->dev));
  const int64_t G = c->n_gates, NB = c->bins.n_bins;
  TRY(ensure(c, c->rep_small, 64));
  double* d_tot = ptr<double>(c->rep_small);                                           // [4]
  unsigned long long* d_tmax = reinterpret_cast<unsigned long long*>(d_tot + 4);       // [1]
  uint32_t* d_peak = reinterpret_cast<uint32_t*>(d_tot + 5);                           // [1]
  TRY(fill_u64(c, c->rep_small.p, 8, 0ull));
  TRY(gate_prep(c, net_load_ff, leak_scale, kAnyMfix));
  if (G > 0) TRY(fill_u64(c, gate_energy_fj, 4 * G, 0ull));
  if (c->n_blocks > 0) {
    ReportArgs a;
    a.ev = ev_view(c);
    a.plan = ptr<uint2>(c->plan_blk);
    a.gprep = ptr<GatePrep>(c->gprep);
    a.lib = lib_view(c);
    a.lut = lut_args(c, kAnyMfix);
    a.bins = c->bins;
    a.glitch_clk = c->par.glitch_clk_ps;
    a.ge = gate_energy_fj;
    a.t_max = d_tmax;
    LAUNCH(c, "k_gate_report", k_gate_report, dim3(grid_for(c->n_blocks, kFwdThreads)), dim3(kFwdThreads),
           lib_lds_bytes(c), a);
  }
  if (G > 0) {
    const LibView L = lib_view(c);
    LAUNCH(c, "k_report_finalize", k_report_finalize, dim3(grid_for(G, 256)), dim3(256), 0,
           (const GatePrep*)ptr<GatePrep>(c->gprep), L.meta, L.leak, L.wide, c->all_pins, G, c->bins.t_end,
           gate_energy_fj, d_tot);
  }
  if (power_mw && NB > 0)
    LAUNCH(c, "k_peak", k_peak, dim3((unsigned)std::min<int64_t>(grid_for(NB, 256), 4096)), dim3(256), 0, power_mw,
           NB, d_peak);
  double h[6] = {0, 0, 0, 0, 0, 0};
  HIPCHK(c, hipMemcpyAsync(h, c->rep_small.p, sizeof h, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  uint64_t tm = 0;
  uint32_t pk = 0;
  memcpy(&tm, &h[4], 8);
  memcpy(&pk, &h[5], 4);
  const bool has_ev = c->ev.n_events > 0;
  const double t_max = has_ev ? (double)tm : -1.0;
  const double nan = std::nan("");
  for (int k = 0; k < 4; ++k) totals[k] = h[k];
  totals[4] = t_max;
  if (power_mw && NB > 0) {
    const uint32_t u = (pk & 0x80000000u) ? (pk & 0x7fffffffu) : ~pk;
    float f;
    memcpy(&f, &u, 4);
    totals[5] = f;
  } else {
    totals[5] = nan;
  }
  for (int k = 0; k < 4; ++k) totals[6 + k] = t_max > 0 ? h[k] / t_max : nan;
  totals[10] = (h[0] + h[1] + h[2] + h[3]) / (double)c->bins.t_end;
  totals[11] = (double)c->bins.t_end;
  return GTP_OK;
}

gtp_status gtp_debug_event_trace(gtp_ctx c, int32_t* state_before, int64_t* bin) {
  TRY(need(c, true, true, true, true));
  if (c->ev.n_events == 0) return GTP_OK;
  if (!state_before || !bin) return fail(c, GTP_ERR_INVALID_ARG, "null trace output");
  HIPCHK(c, hipSetDevice(c->dev));
  const int64_t N = c->ev.n_events;
  // any loads: the trace does not depend on them; the gate preparation needs a net-load array
  TRY(ensure(c, c->adj_w, (size_t)(c->n_nets + 2) * 4));
  TRY(fill_u64(c, c->adj_w.p, (c->n_nets + 1) / 2 + 1, 0x3f8000003f800000ull));
  if (c->tun.algo == 0) {
    // the packed path's own state tracking, done once when the layout is
    // built: the layout is rebuilt with the trace written alongside; events
    // it does not pack keep -1
    LAUNCH(c, "k_fill_i32", k_fill_i32, dim3(grid_for(N, 256)), dim3(256), 0, state_before, N, -1);
    TRY(fill_u64(c, bin, N, ~0ull));
    drop_pack(c);
    TRY(pack_for(c, c->ev, c->plan_blk, c->bins, c->pk, c->pack_ms, state_before, bin));
    c->pack_ok = true;
    return GTP_OK;
  }
  TRY(gate_prep(c, ptr<float>(c->adj_w), nullptr, kAnyMfix));
  TraceArgs a;
  a.ev = ev_view(c);
  a.plan = ptr<uint2>(c->plan_blk);
  a.gprep = ptr<GatePrep>(c->gprep);
  a.lib = lib_view(c);
  a.lut = lut_args(c, kAnyMfix);
  a.bins = c->bins;
  a.state = state_before;
  a.bin = bin;
  LAUNCH(c, "k_event_trace", k_event_trace, dim3(grid_for(c->n_blocks, kFwdThreads)), dim3(kFwdThreads), lib_lds_bytes(c), a);
  return GTP_OK;
}

}  // extern "C"

extern "C" {

gtp_status gtp_profile_enable(gtp_ctx c, int enable) {
  if (!c) return GTP_ERR_INVALID_ARG;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  prof_clear(c);
  c->prof_names.clear();
  c->prof_on = enable != 0;
  return GTP_OK;
}

gtp_status gtp_profile_read(gtp_ctx c, int32_t cap, const char** names, int64_t* launches, double* total_ms,
                            int32_t* n_out) {
  if (!c || !n_out || cap < 0 || (cap > 0 && (!names || !launches || !total_ms))) return GTP_ERR_INVALID_ARG;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const int n = (int)c->prof_names.size();
  std::vector<double> ms(n, 0.0);
  std::vector<int64_t> cnt(n, 0);
  for (const auto& r : c->prof_recs) {
    float t = 0.f;
    HIPCHK(c, hipEventElapsedTime(&t, r.a, r.b));
    ms[r.id] += t;
    cnt[r.id] += 1;
  }
  const int m = std::min(n, (int)cap);
  for (int i = 0; i < m; ++i) {
    names[i] = c->prof_names[i].c_str();
    launches[i] = cnt[i];
    total_ms[i] = ms[i];
  }
  *n_out = n;
  return GTP_OK;
}

// ---- streamed windows (chunked evaluation of a long trace) ----------------

}  // extern "C"

namespace {
// Evaluates the window held by slot sl: times made relative to its start, its
// lane-block plan, the forward into its bins of the trace's power array, then
// the pin values every gate carries out of it (into the netlist's initial
// values, which the next window starts from).
template <class Slot>
gtp_status stream_window(gtp_ctx c, Slot& sl, const float* net_load_ff, const float* leak_scale, float* power_mw) {
  if (sl.n > 0)
    LAUNCH(c, "k_shift_times", k_shift_times, dim3(grid_for(sl.n, 256)), dim3(256), 0, ptr<int64_t>(sl.t), sl.n, sl.t0);
  gtp_events ev;
  ev.n_events = sl.n;
  ev.t_end_ps = sl.t1 - sl.t0;
  ev.gate_off = ptr<int64_t>(sl.gate_off);
  ev.t_ps = ptr<int64_t>(sl.t);
  ev.pin_bit = ptr<uint8_t>(sl.pb);
  ev.slew_ps = ptr<float>(sl.slew);
  c->ev = ev;
  c->ev_ok = false;
  drop_pack(c);
  TRY(build_block_plan(c));
  c->ev_ok = true;
  c->bins = bins_for(c, ev.t_end_ps);
  if (c->st_validate) TRY(validate_events(c, ev, c->plan_blk, c->n_blocks));
  TRY(gtp_forward(c, net_load_ff, leak_scale, power_mw + sl.t0 / c->par.bin_ps));
  if (c->n_blocks > 0)
    LAUNCH(c, "k_stream_carry", k_stream_carry, dim3(grid_for(c->n_blocks, kFwdThreads)), dim3(kFwdThreads), 0,
           ev_view(c), (const uint2*)ptr<uint2>(c->plan_blk), ptr<uint32_t>(c->gate_init));
  return GTP_OK;
}
}  // namespace

extern "C" {

gtp_status gtp_stream_begin(gtp_ctx c, int64_t t_end_ps, int32_t validate) {
  TRY(need(c, true, true, false, true));
  if (t_end_ps < 1 || (validate != 0 && validate != 1))
    return fail(c, GTP_ERR_INVALID_ARG, "stream of %lld ps, validate %d", (long long)t_end_ps, validate);
  HIPCHK(c, hipSetDevice(c->dev));
  if (!c->copy_stream) HIPCHK(c, hipStreamCreateWithFlags(&c->copy_stream, hipStreamNonBlocking));
  for (auto& sl : c->st_slot) {
    if (!sl.copied) HIPCHK(c, hipEventCreateWithFlags(&sl.copied, hipEventDisableTiming));
    if (!sl.done) HIPCHK(c, hipEventCreateWithFlags(&sl.done, hipEventDisableTiming));
    sl.used = false;
  }
  c->ev_ok = false;
  drop_pack(c);
  drop_graph(c);
  const size_t gb = (size_t)std::max<int64_t>(c->n_gates, 1) * 4;
  TRY(ensure(c, c->st_init, gb));
  HIPCHK(c, hipMemcpyAsync(c->st_init.p, c->gate_init.p, gb, hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->st_on = true;
  c->st_validate = validate;
  c->st_end = t_end_ps;
  c->st_next_push = c->st_next_step = 0;
  c->st_head = c->st_pending = 0;
  return GTP_OK;
}

gtp_status gtp_stream_push(gtp_ctx c, const gtp_events* ev, int64_t t0_ps, int64_t t1_ps) {
  if (!c || !ev) return GTP_ERR_INVALID_ARG;
  if (!c->st_on) return fail(c, GTP_ERR_NOT_LOADED, "no stream open (gtp_stream_begin)");
  if (c->st_pending >= 2) return fail(c, GTP_ERR_INVALID_ARG, "two windows are pending: gtp_stream_step first");
  const int64_t D = c->par.bin_ps, clk = c->par.glitch_clk_ps;
  if (t0_ps != c->st_next_push || t1_ps <= t0_ps || t1_ps > c->st_end)
    return fail(c, GTP_ERR_INVALID_ARG, "window [%lld, %lld): windows must tile [0, %lld) in order (next starts at %lld)",
                (long long)t0_ps, (long long)t1_ps, (long long)c->st_end, (long long)c->st_next_push);
  if (t0_ps % D != 0 || (t1_ps % D != 0 && t1_ps != c->st_end))
    return fail(c, GTP_ERR_INVALID_ARG, "window cuts must be multiples of the %lld ps bin", (long long)D);
  if (clk > 0 && (t0_ps % clk != 0 || (t1_ps % clk != 0 && t1_ps != c->st_end)))
    return fail(c, GTP_ERR_INVALID_ARG, "window cuts must be multiples of the %lld ps glitch clock", (long long)clk);
  const int64_t N = ev->n_events, G = c->n_gates;
  if (N < 0 || !ev->gate_off || (N > 0 && (!ev->t_ps || !ev->pin_bit || !ev->slew_ps)))
    return fail(c, GTP_ERR_INVALID_ARG, "window event arrays");
  if (ev->gate_off[0] != 0 || ev->gate_off[G] != N)
    return fail(c, GTP_ERR_INVALID_ARG, "window gate_off must run from 0 to n_events");
  for (int64_t g = 0; g < G; ++g)
    if (ev->gate_off[g + 1] < ev->gate_off[g]) return fail(c, GTP_ERR_INVALID_ARG, "window gate_off decreases at %lld",
                                                          (long long)g);
  HIPCHK(c, hipSetDevice(c->dev));
  auto& sl = c->st_slot[(c->st_head + c->st_pending) % 2];
  if (sl.used) HIPCHK(c, hipEventSynchronize(sl.done));   // the window that last used the slot is done
  TRY(ensure(c, sl.gate_off, (size_t)(G + 1) * 8));
  TRY(ensure(c, sl.t, (size_t)std::max<int64_t>(N, 1) * 8));
  TRY(ensure(c, sl.pb, (size_t)((std::max<int64_t>(N, 1) + 15) & ~(int64_t)15)));
  TRY(ensure(c, sl.slew, (size_t)std::max<int64_t>(N, 1) * 4));
  HIPCHK(c, hipMemcpyAsync(sl.gate_off.p, ev->gate_off, (size_t)(G + 1) * 8, hipMemcpyHostToDevice, c->copy_stream));
  if (N > 0) {
    HIPCHK(c, hipMemcpyAsync(sl.t.p, ev->t_ps, (size_t)N * 8, hipMemcpyHostToDevice, c->copy_stream));
    HIPCHK(c, hipMemcpyAsync(sl.pb.p, ev->pin_bit, (size_t)N, hipMemcpyHostToDevice, c->copy_stream));
    HIPCHK(c, hipMemcpyAsync(sl.slew.p, ev->slew_ps, (size_t)N * 4, hipMemcpyHostToDevice, c->copy_stream));
  }
  HIPCHK(c, hipEventRecord(sl.copied, c->copy_stream));
  sl.n = N;
  sl.t0 = t0_ps;
  sl.t1 = t1_ps;
  c->st_pending += 1;
  c->st_next_push = t1_ps;
  return GTP_OK;
}

gtp_status gtp_stream_step(gtp_ctx c, const float* net_load_ff, const float* leak_scale, float* power_mw) {
  if (!c) return GTP_ERR_INVALID_ARG;
  if (!c->st_on) return fail(c, GTP_ERR_NOT_LOADED, "no stream open (gtp_stream_begin)");
  if (c->st_pending == 0) return fail(c, GTP_ERR_INVALID_ARG, "no window pushed");
  if (!net_load_ff || !power_mw) return fail(c, GTP_ERR_INVALID_ARG, "null stream argument");
  HIPCHK(c, hipSetDevice(c->dev));
  auto& sl = c->st_slot[c->st_head];
  // the caller's host arrays are free once the copy is done
  HIPCHK(c, hipEventSynchronize(sl.copied));
  HIPCHK(c, hipStreamWaitEvent(c->stream, sl.copied, 0));
  c->st_inside = true;
  const gtp_status st = stream_window(c, sl, net_load_ff, leak_scale, power_mw);
  c->st_inside = false;
  if (st != GTP_OK) {
    // the carried values are no longer those of a window boundary: end the stream
    (void)gtp_stream_end(c);
    return st;
  }
  HIPCHK(c, hipEventRecord(sl.done, c->stream));
  sl.used = true;
  c->st_head = (c->st_head + 1) % 2;
  c->st_pending -= 1;
  c->st_next_step = sl.t1;
  return GTP_OK;
}

gtp_status gtp_stream_end(gtp_ctx c) {
  if (!c) return GTP_ERR_INVALID_ARG;
  if (!c->st_on) return GTP_OK;
  HIPCHK(c, hipSetDevice(c->dev));
  if (c->copy_stream) HIPCHK(c, hipStreamSynchronize(c->copy_stream));
  const size_t gb = (size_t)std::max<int64_t>(c->n_gates, 1) * 4;
  HIPCHK(c, hipMemcpyAsync(c->gate_init.p, c->st_init.p, gb, hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->st_on = false;
  c->st_pending = 0;
  c->ev_ok = false;
  drop_pack(c);
  return GTP_OK;
}

}  // extern "C"
