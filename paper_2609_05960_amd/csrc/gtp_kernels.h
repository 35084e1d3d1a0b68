// Kernels of the binned power-waveform library (gfx950, wave64).
//
// Work decomposition. The gate-major event array is cut into lane blocks of
// kLaneEvents consecutive events. One lane walks one block in order, so the
// gate state is a running register (each event toggles one pin: the state is
// the gate's initial bits XOR the parity of the toggles seen so far). A block
// may hold the tail of one gate and many short gates (sparse gates are packed)
// or a slice of one long gate (dense gates are cut into many blocks), so work
// per lane is fixed whatever the per-gate event counts. The plan gives every
// block its first gate and the toggle parity that gate carries into the block.
//
// Order of operations per event follows Algorithm 1 (Sec. 4.3): the events of
// one gate that share a timestamp are looked up with the state before the
// group, then applied; leakage is charged in the step form described in
// gtp_device.h.
#pragma once
#include "gtp_device.h"
#include "gtp_scan.h"

namespace gtp {

// Lookup and energy of one event (shared by every path so results agree bit
// for bit). Updates the running quantised leakage rate q_cur.
struct GateCtx {
  GatePrep gp;
  CellMeta cm;
  uint32_t in_mask;     // the pins of the state index (inputs, or every pin)
  int32_t n_state;      // pins below n_state change the state (n_in or n_in + 1)
  int32_t q_cur;
};

__device__ __forceinline__ void gate_begin(GateCtx& G, const GatePrep* __restrict__ gprep, const LdsLib& L, int64_t g,
                                           uint32_t par, float rate_scale) {
  const int4* src = reinterpret_cast<const int4*>(gprep + g);
  int4 a = src[0], b = src[1];
  G.gp.cell = a.x; G.gp.init = (uint32_t)a.y; G.gp.jq = a.z; G.gp.beta = __int_as_float(a.w);
  G.gp.esw_rise = __int_as_float(b.x); G.gp.esw_fall = __int_as_float(b.y);
  G.gp.lam = __int_as_float(b.z); G.gp.dbeta_dc = __int_as_float(b.w);
  G.cm = L.meta[G.gp.cell];
  G.in_mask = state_mask(G.cm.n_in, L.all_pins);
  G.n_state = G.cm.n_in + L.all_pins;
  const uint32_t s = (G.gp.init ^ par) & G.in_mask;
  G.q_cur = qrate(G.gp.lam, L.leak[leak_entry(L, G.cm, G.gp.cell, s)], rate_scale);
}

struct LutArgs {
  const float4* __restrict__ quads;
  int32_t n_slew, n_load;
  float rate_scale;   // FP32(2^m * 1e-6)
  float two_sh;       // 2^(m-32)
};

__device__ __forceinline__ EventOut event_energy(GateCtx& G, const LdsLib& L, const LutArgs& A, int pin, int v,
                                                 float slew, uint32_t par_gs, uint32_t par) {
  EventOut o;
  const uint32_t s = (G.gp.init ^ par_gs) & G.in_mask;
  const int32_t qb = L.map_q[map_entry(L, G.cm, G.gp.cell, s, (uint32_t)v)];
  int i;
  float alpha;
  slew_segment(L.slew + G.cm.axis_off, L.slew_inv + G.cm.axis_off, A.n_slew, slew, i, alpha);
  const float4 q = A.quads[qb + i * (A.n_load - 1) + G.gp.jq];
  float e = bilerp_quad(q, alpha, G.gp.beta);
  if (pin == G.cm.n_in) e = __fadd_rn(e, v ? G.gp.esw_rise : G.gp.esw_fall);
  int32_t delta = 0;
  if (pin < G.n_state) {
    const uint32_t s_new = (G.gp.init ^ par ^ (1u << pin)) & G.in_mask;
    const int32_t qn = qrate(G.gp.lam, L.leak[leak_entry(L, G.cm, G.gp.cell, s_new)], A.rate_scale);
    delta = qn - G.q_cur;
    G.q_cur = qn;
  }
  o.e = e;
  o.delta = delta;
  o.s = (int32_t)s;
  return o;
}

// ---------------------------------------------------------------------------
// forward, packed tile-major path
// ---------------------------------------------------------------------------
// One workgroup per time tile: the tile's 2^tile_log2 bins (X and S, int64)
// live in LDS, every wavefront takes whole 64-unit groups of the tile (one
// unit per lane, see gtp_pack.h) and accumulates with LDS atomics; at the
// end the tile's bins are stored (each bin belongs to exactly one tile, so
// no global atomics and no zero fill are needed).
struct PackedFwdArgs {
  const uint32_t* ev;        // per event: word, table row, slew weight (3 words)
  const uint2* desc;
  const int64_t* grp_off;
  const int32_t* tile_grp;
  const GateParam* gparam;   // per cell-sorted gate, this call
  LibView lib;
  LutArgs lut;
  BinSpec bins;
  int32_t sw_mode;
  double v2;                 // Vdd^2
  int64_t* X;
  int64_t* S;
  const int4* phases;        // table phases (null: every quad from global memory)
  const int32_t* ph_off;
  int32_t slot_quads;        // quads of one LDS table slot
  long long* tile_tot;       // non-null: S gets the within-tile exclusive prefix of
                             // the steps and tile_tot[tile] their total
  const float* rgl;          // per packed event its energy factor (glitch detection on), else null
};

// LDS of the packed kernels: the library's meta + leakage prefix, then the
// tile's bins (two int64 per bin), then two table slots of slot_quads quads
// (as many as the remaining LDS holds, a multiple of 64).
// (36 words between the library prefix and the bins: the in-tile prefix scan's
// wavefront sums)
constexpr int kScanScratchWords = 36;
__device__ __host__ __forceinline__ size_t packed_bins_word_offset(int32_t lib_words) {
  return (size_t)((lib_words + 3) & ~3) + kScanScratchWords;
}

// One wavefront group's data in registers: unit descriptor, gate
// parameters and the lane's event records (k-major positions resolved).
template <int kS>
struct GroupRegs {
  uint2 d;
  GateParam gp;
  int len;
  int kmax;
  uint32_t wv[kS];
  uint32_t rv[kS];
  float av[kS];
  float gv[kS];   // energy factors (glitch detection on only)
};

// A unit descriptor loaded non-temporally (the adjoint reads each once).
typedef unsigned int desc_vec __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint2 desc_nt(const uint2* p) {
  const desc_vec v = __builtin_nontemporal_load(reinterpret_cast<const desc_vec*>(p));
  return make_uint2(v.x, v.y);
}

// Issue every load of one group (descriptor and offset already loaded).
// With mine false the lane's length still counts for the positions of the
// other lanes, but its own loads are skipped.
// kS is the longest unit the layout holds (its unit_events), 8 or 16; kGl:
// the events' energy factors are loaded too (glitch detection on); kNt: the
// records load non-temporally (read once: their lines leave the L2 first, so
// that the gathered lines that are read again, bin weights and gate records,
// stay; the adjoint runs about 2 % faster with it, the forward not measurably).
template <int kS, bool kGl, bool kNt = false>
__device__ __forceinline__ void group_issue(const PackedFwdArgs& a, uint2 d, int64_t off, GroupRegs<kS>& G,
                                            bool mine = true) {
  G.d = d;
  const bool valid = d.x != 0xffffffffu;
  G.len = valid ? (int)(d.x >> 28) + 1 : 0;
  // no else branch: a lane without a unit (len 0) gathers record 0 and never
  // uses it, and nothing reads the loaded registers before the group is
  // processed (a select on them would wait for the load right here)
  if (mine) G.gp = a.gparam[valid ? (d.x & 0x0fffffffu) : 0u];
  // the offset is the same on every lane: keep it scalar so the loads use a
  // scalar base and a 32-bit lane offset
  const int64_t offu = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(off >> 32)) << 32) |
                                 (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int32_t)off));
  // the group's events: word, row and slew weight of each, 12 bytes
  const uint3* __restrict__ ep = reinterpret_cast<const uint3*>(a.ev) + offu;
  uint32_t o = 0;
  G.kmax = 0;
  // slot kk holds event kk of every lane longer than kk; slots past the
  // longest unit are skipped by a wave-uniform branch
#pragma unroll
  for (int kk = 0; kk < kS; ++kk) {
    const bool on = G.len > kk;
    const uint64_t m = __ballot(on);
    if (m != 0) {
      G.kmax = kk + 1;
      if (on && mine) {
        const uint32_t r =
            o + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
        uint3 v;
        if (kNt) {
          const uint32_t* vp = reinterpret_cast<const uint32_t*>(ep + r);
          v.x = __builtin_nontemporal_load(vp);
          v.y = __builtin_nontemporal_load(vp + 1);
          v.z = __builtin_nontemporal_load(vp + 2);
        } else {
          v = ep[r];
        }
        G.wv[kk] = v.x;
        G.rv[kk] = v.y;
        G.av[kk] = __uint_as_float(v.z);
        if (kGl) G.gv[kk] = a.rgl[offu + r];
      }
      o += (uint32_t)__popcll(m);
    }
  }
}

// Table quad of a lane's event: from the phase's LDS slot when the quad lies
// in its range [lo, lo + n), else from global memory. The slot read is
// unconditional (clamped index) through an LDS pointer and the global read is
// predicated, so the two stay an LDS and a global load rather than being
// merged into one flat load.
// (The fallback is a non-temporal load: it differs from the slot load, so the
// optimiser cannot sink the two into one load through a selected pointer.)
typedef float quad_vec __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) quad_vec lds_float4;

__device__ __forceinline__ const lds_float4* lds_ptr(const float4* p) { return (const lds_float4*)p; }

__device__ __forceinline__ float4 quad_at(const float4* __restrict__ quads, const lds_float4* slot, uint32_t lo,
                                          uint32_t n, uint32_t qi) {
  const uint32_t li = qi - lo;
  const bool in = li < n;
  quad_vec v = slot[in ? li : 0u];
  if (!in) v = __builtin_nontemporal_load(reinterpret_cast<const quad_vec*>(quads) + qi);
  return make_float4(v.x, v.y, v.z, v.w);
}

// Table quad of a lane's event when the phase's slot holds every quad its
// groups read (index clamped into the slot, so a stray index stays in LDS;
// n is at least 1 whenever a group of the phase holds an event).
__device__ __forceinline__ float4 quad_slot(const lds_float4* slot, uint32_t lo, uint32_t n, uint32_t qi) {
  const quad_vec v = slot[min(qi - lo, n - 1u)];
  return make_float4(v.x, v.y, v.z, v.w);
}

// Accumulates one group (loaded into G) into the tile's LDS bins. The table
// quad and the leakage value after event k+1 load into one buffer while event
// k is accumulated from the other. With kSlotOnly every quad comes from the
// slot and the function issues no global load, so the next group's loads
// stay in flight while this group is accumulated.
template <int kS, bool kSlotOnly, bool kGl>
__device__ __forceinline__ void process_group(const PackedFwdArgs& a, const LdsLib& L, const GroupRegs<kS>& G,
                                              unsigned long long* xs, unsigned long long* ss, const lds_float4* slot,
                                              uint32_t lo, uint32_t n) {
  const BinSpec& B = a.bins;
  const uint32_t rmask = (1u << B.r_bits) - 1u;
  const int32_t D32 = (int32_t)B.D;
  const float4* __restrict__ quads = a.lut.quads;
  const int len = G.len;
  const GateParam gp = G.gp;
  const int cell = (int)(G.d.y >> 16);
  const UnitLut u = unit_lut(L, a.lut.n_load, cell, gp.C, a.v2, a.sw_mode);
  const uint32_t jq = u.jq;
  const CellMeta cm = L.meta[cell];
  const float* lk = L.leak + cm.leak_off;
  // desc.y low half: the pin values (a kCellDirect cell, masked to its state)
  // or the leakage item (wider cells, below 256) before the unit
  int32_t q_cur = qrate(gp.lam, lk[G.d.y & 0xffffu & state_mask(cm.n_in, L.all_pins)], a.lut.rate_scale);
  struct Pre {
    float4 q;        // table quad
    float lk_after;  // leakage value of the input state after the event
  };
  auto prefetch = [&](int k, Pre& P) {
    const uint32_t qi = (G.rv[k] & kRowMask) + jq;
    P.q = kSlotOnly ? quad_slot(slot, lo, n, qi) : quad_at(quads, slot, lo, n, qi);
    P.lk_after = lk[G.wv[k] >> kStateShift];
  };
  Pre pre[2];
  if (len > 0) prefetch(0, pre[0]);
#pragma unroll
  for (int kk = 0; kk < kS; ++kk) {
    if (kk < G.kmax && len > kk) {
      const uint32_t w = G.wv[kk];
      const uint32_t rv = G.rv[kk];
      if (kk + 1 < kS && len > kk + 1) prefetch(kk + 1, pre[(kk + 1) & 1]);
      const Pre& P = pre[kk & 1];
      float e = bilerp_quad(P.q, G.av[kk], u.beta);
      if (rv & (1u << kOutBit)) e = __fadd_rn(e, (rv >> 31) ? u.esw_rise : u.esw_fall);
      if (kGl) e = __fmul_rn(e, G.gv[kk]);
      int64_t x = energy_fixed(e, a.lut.two_sh);
      const uint32_t tl = w & kTimeMask;
      const uint32_t bl = tl >> B.r_bits;
      // leakage step: an output event leaves the input state (and so the
      // rate) unchanged, so dq = 0 for it without a branch
      const int32_t qn = qrate(gp.lam, P.lk_after, a.lut.rate_scale);
      const int32_t dq = qn - q_cur;
      q_cur = qn;
      x += (int64_t)dq * (int64_t)(D32 - (int32_t)(tl & rmask));
      if (dq != 0) atomicAdd(&ss[bl], (unsigned long long)(int64_t)dq);
      atomicAdd(&xs[bl], (unsigned long long)x);
    }
  }
}

// Table-phase state of one workgroup (see fwd_tile_body).
struct PhaseState {
  int32_t ph, ph1;     // current phase, end of the tile's phases
  int64_t ge;          // end group of the current phase
  uint32_t lo, n;      // its quad range
};

__device__ __forceinline__ void phase_enter(const PackedFwdArgs& a, PhaseState& P, int64_t g0) {
  const int4 Q = a.phases[P.ph];
  P.ge = g0 + Q.x;
  P.lo = (uint32_t)Q.y;
  P.n = (uint32_t)Q.z;
}

// Quads [lo, lo + n) of the table array into an LDS slot, by direct
// global-to-LDS loads: wavefront w copies 64-quad chunks w, w + nwave, ...
// (a lane past n re-reads the last quad; the slot holds whole chunks). The
// copy completes at the issuing wavefront's next vmcnt(0) wait.
template <int kThreads>
__device__ __forceinline__ void slot_fill(const float4* __restrict__ quads, uint32_t lo, uint32_t n, float4* slot) {
  constexpr int nwave = kThreads / 64;
  const int lane = (int)(threadIdx.x & 63);
  const int chunks = (int)((n + 63) >> 6);
  for (int c = (int)(threadIdx.x >> 6); c < chunks; c += nwave) {
    const uint32_t i = min((uint32_t)(c * 64 + lane), n - 1u);
    __builtin_amdgcn_global_load_lds((const void*)(quads + lo + i),
                                     (__attribute__((address_space(3))) void*)(slot + c * 64), 16, 0, 0);
  }
}

__device__ __forceinline__ void wait_vmem() { __builtin_amdgcn_s_waitcnt(0x0F70); }  // vmcnt(0)

// Boundary ph -> ph + 1, taken by every wavefront: wait for this wavefront's
// share of the next phase's quads, one barrier (after it the slot is whole
// and the previous phase's slot is free), then the following phase's quads
// start loading into that free slot.
template <int kThreads>
__device__ __forceinline__ void phase_advance(const PackedFwdArgs& a, PhaseState& P, float4* slots, int64_t g0) {
  wait_vmem();
  __syncthreads();
  ++P.ph;
  phase_enter(a, P, g0);
  if (P.ph + 1 < P.ph1) {
    const int4 Q = a.phases[P.ph + 1];
    slot_fill<kThreads>(a.lut.quads, (uint32_t)Q.y, (uint32_t)Q.z, slots + ((P.ph + 1) & 1) * a.slot_quads);
  }
}

// One time tile of one trace: the tile's bins are zeroed in LDS, every
// wavefront takes whole groups of the tile, and the bins are stored at the
// end (each bin belongs to exactly one tile). Memory-level parallelism: a
// wavefront works on group i while the loads of group i+1 (gate parameters,
// events) and the descriptors of group i+2 are in flight; the loop alternates
// two register buffers, so nothing is copied between groups.
//
// Table phases (slots non-null and the tile has phases): the tile's groups
// are cut into phases whose cells' table quads fit one LDS slot. Phase p reads
// slot p & 1; while it runs, phase p+1's quads load straight into the other
// slot, and one barrier at the boundary separates the phases. Every
// wavefront crosses every boundary once, in order, whether or not it has
// groups in a phase.
template <int kThreads, int kS, bool kSlotOnly, bool kGl>
__device__ __forceinline__ void fwd_tile_body(const PackedFwdArgs& a, const LdsLib& L, unsigned long long* xs,
                                              unsigned long long* ss, int32_t tile, float4* slots) {
  const BinSpec& B = a.bins;
  const int nb = 1 << B.tile_log2;
  for (int i = threadIdx.x; i < 2 * nb; i += kThreads) xs[i] = 0ull;
  // without phases every quad comes from global memory; the slot reads of
  // quad_at then touch the bins (any valid LDS address) and are discarded
  float4* const lds_slots = slots ? slots : reinterpret_cast<float4*>(xs);
  const int64_t g0 = a.tile_grp[tile];
  const int64_t g1 = a.tile_grp[tile + 1];
  const int lane = (int)(threadIdx.x & 63);
  constexpr int nwave = kThreads / 64;
  int64_t gi = g0 + (int64_t)(threadIdx.x >> 6);
  // ---- table phases
  PhaseState P;
  P.ph = 0;
  P.ph1 = 0;
  if (slots && a.phases) {
    P.ph = a.ph_off[tile];
    P.ph1 = a.ph_off[tile + 1];
  }
  P.ge = g1;
  P.lo = 0;
  P.n = 0;
  if (P.ph < P.ph1) {
    phase_enter(a, P, g0);
    slot_fill<kThreads>(a.lut.quads, P.lo, P.n, slots + (P.ph & 1) * a.slot_quads);
    wait_vmem();  // the first phase's slot is whole at the barrier below
    if (P.ph + 1 < P.ph1) {
      const int4 Q = a.phases[P.ph + 1];
      slot_fill<kThreads>(a.lut.quads, (uint32_t)Q.y, (uint32_t)Q.z, slots + ((P.ph + 1) & 1) * a.slot_quads);
    }
  }
  GroupRegs<kS> ga, gb;
  uint2 dn = make_uint2(0xffffffffu, 0u);
  int64_t offn = 0;
  // issue the loads of group g into R and prefetch the descriptor of g + nwave
  // the descriptor and offset of group g: unconditional loads, clamped to
  // the tile's last group (a conditional load would make the compiler copy
  // the register at the join, and the copy waits for the load)
  auto load_desc = [&](int64_t g) {
    const int64_t gn = min(g, g1 - 1);
    dn = a.desc[gn * kGroupUnits + lane];
    offn = a.grp_off[gn];
  };
  if (gi < g1) {
    load_desc(gi);
    wait_vmem();
    group_issue<kS, kGl>(a, dn, offn, ga);
    load_desc(gi + nwave);
  }
  __syncthreads();
  // Each step first waits for everything this wavefront has loaded (the
  // current group's records and the next descriptor, issued one group ago),
  // then issues the next group's loads and accumulates the current group.
  // An explicit wait here keeps the compiler from placing its own: it cannot
  // count the group's loads (their number varies), so any wait it derived
  // inside the accumulation would drain the next group's loads as well.
  while (gi < g1) {
    while (gi >= P.ge) phase_advance<kThreads>(a, P, slots, g0);
    wait_vmem();
    if (gi + nwave < g1) group_issue<kS, kGl>(a, dn, offn, gb);
    load_desc(gi + 2 * nwave);
    process_group<kS, kSlotOnly, kGl>(a, L, ga, xs, ss, lds_ptr(lds_slots + (P.ph & 1) * a.slot_quads), P.lo, P.n);
    gi += nwave;
    if (gi >= g1) break;
    while (gi >= P.ge) phase_advance<kThreads>(a, P, slots, g0);
    wait_vmem();
    if (gi + nwave < g1) group_issue<kS, kGl>(a, dn, offn, ga);
    load_desc(gi + 2 * nwave);
    process_group<kS, kSlotOnly, kGl>(a, L, gb, xs, ss, lds_ptr(lds_slots + (P.ph & 1) * a.slot_quads), P.lo, P.n);
    gi += nwave;
  }
  while (P.ph + 1 < P.ph1) phase_advance<kThreads>(a, P, slots, g0);  // boundaries after this wavefront's last group
  __syncthreads();
  if (a.tile_tot) {
    // exclusive prefix of the tile's steps, in place: thread i takes a run of
    // consecutive bins, the runs' sums are scanned over the wavefronts
    long long* ws = reinterpret_cast<long long*>(xs) - kScanScratchWords / 2;
    const int per = (nb + kThreads - 1) / kThreads;
    const int i0 = min((int)threadIdx.x * per, nb), i1 = min(i0 + per, nb);
    long long sum = 0;
    for (int i = i0; i < i1; ++i) sum += (long long)ss[i];
    long long inc = sum;
    for (int o = 1; o < 64; o <<= 1) {
      const long long t = __shfl_up(inc, o, 64);
      if (lane >= o) inc += t;
    }
    const int wave = (int)(threadIdx.x >> 6);
    if (lane == 63) ws[wave] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
      long long acc = 0;
      for (int w = 0; w < nwave; ++w) {
        const long long t = ws[w];
        ws[w] = acc;
        acc += t;
      }
      a.tile_tot[tile] = acc;
    }
    __syncthreads();
    long long run = ws[wave] + inc - sum;
    for (int i = i0; i < i1; ++i) {
      const long long v = (long long)ss[i];
      ss[i] = (unsigned long long)run;
      run += v;
    }
    __syncthreads();
  }
  const int64_t b0 = (int64_t)tile << B.tile_log2;
  for (int i = threadIdx.x; i < nb; i += kThreads) {
    if (b0 + i < B.n_bins) {
      a.X[b0 + i] = (int64_t)xs[i];
      a.S[b0 + i] = (int64_t)ss[i];
    }
  }
}

// One workgroup per time tile of a single trace. kSlotOnly: every table phase
// holds all the quads of its groups (the host launches it only then); kGl:
// glitch detection on (each event's energy times its factor).
template <int kThreads, int kS, bool kSlotOnly, bool kGl>
__global__ void __launch_bounds__(kThreads) k_fwd_packed(PackedFwdArgs a) {
  extern __shared__ uint32_t lds[];
  const LdsLib L = stage_library_ml(a.lib, lds);
  unsigned long long* xs = reinterpret_cast<unsigned long long*>(lds + packed_bins_word_offset(a.lib.lds_words_ml));
  unsigned long long* ss = xs + (1 << a.bins.tile_log2);
  float4* slots = a.phases ? reinterpret_cast<float4*>(ss + (1 << a.bins.tile_log2)) : nullptr;
  // one tile per workgroup; past the largest grid (a dispatch holds at most
  // 2^32 work-items) the workgroups take further tiles in turn
  for (int64_t tile = blockIdx.x; tile < a.bins.n_tiles; tile += gridDim.x) {
    if (tile != blockIdx.x) __syncthreads();   // the previous tile is done with the LDS
    fwd_tile_body<kThreads, kS, kSlotOnly, kGl>(a, L, xs, ss, (int32_t)tile, slots);
  }
}

// ---------------------------------------------------------------------------
// batched traces: one persistent launch over all (trace, tile) work items
// ---------------------------------------------------------------------------
struct TraceDev {
  const uint32_t* ev;
  const float* rgl;
  const int4* phases;
  const int32_t* ph_off;
  int32_t slot_quads;
  const uint2* desc;
  const int64_t* grp_off;
  const int32_t* tile_grp;
  BinSpec bins;
  int64_t bin_off;   // first bin of the trace in the concatenated bins
  int64_t tile_off;  // first tile of the trace in the concatenated tiles
};

struct BatchFwdArgs {
  PackedFwdArgs base;          // shared fields: gate parameters, library, LUT, switching mode
  const TraceDev* traces;
  const int2* items;           // (trace, tile), largest first
  int64_t n_items;
  int64_t* X;                  // concatenated bins
  int64_t* S;                  // within-tile exclusive prefix of the leakage steps
  long long* tile_tot;         // per concatenated tile: total leakage step
};

// One workgroup per work item (trace, tile): the items are listed largest
// first, so the hardware's in-order dispatch hands out the long tiles first
// and the short ones fill in at the end. Each workgroup reads its item once,
// with a uniform index, so the trace record stays in scalar registers.
// kSlotOnly: every trace has table phases that hold all their groups' quads.
template <int kThreads, int kS, bool kSlotOnly, bool kGl>
__global__ void __launch_bounds__(kThreads) k_fwd_batched(BatchFwdArgs a) {
  extern __shared__ uint32_t lds[];
  const LdsLib L = stage_library_ml(a.base.lib, lds);
  const int2 w = a.items[blockIdx.x];
  const TraceDev T = a.traces[w.x];
  PackedFwdArgs p = a.base;
  p.ev = T.ev;
  p.rgl = T.rgl;
  p.desc = T.desc;
  p.grp_off = T.grp_off;
  p.tile_grp = T.tile_grp;
  p.bins = T.bins;
  p.X = a.X + T.bin_off;
  p.S = a.S + T.bin_off;
  p.phases = T.phases;
  p.ph_off = T.ph_off;
  p.slot_quads = T.slot_quads;
  p.tile_tot = a.tile_tot ? a.tile_tot + T.tile_off : nullptr;
  unsigned long long* xs = reinterpret_cast<unsigned long long*>(lds + packed_bins_word_offset(a.base.lib.lds_words_ml));
  unsigned long long* ss = xs + (1 << T.bins.tile_log2);
  float4* slots = T.phases ? reinterpret_cast<float4*>(ss + (1 << T.bins.tile_log2)) : nullptr;
  fwd_tile_body<kThreads, kS, kSlotOnly, kGl>(p, L, xs, ss, w.y, slots);
}

// Per-call gate records (output load, leakage scale) in cell-sorted order,
// plus each block's sum of its gates' quantised initial leakage rates
// (l0_part[block]; their total is L0, summed by the kernel that needs it).
struct GateParamArgs {
  const int32_t* gperm;      // sorted index -> gate (for the caller's leakage scales)
  const int32_t* gcell;      // sorted index -> cell
  const int32_t* gout;       // sorted index -> output net
  const uint32_t* ginit;     // sorted index -> initial pin values
  const float* net_load;
  const float* leak_scale;   // may be null (all 1)
  const CellMeta* meta;
  const float* leak;
  WideView wide;             // cells with more than 8 state pins
  int64_t n_gates;
  float rate_scale;
  float max_scale;
  float load_cap;            // loads must lie in [0, load_cap]
  int32_t all_pins;          // state index over every pin
  GateParam* out;
  long long* l0_part;        // [blocks]
  int32_t* flag;             // bit 0: a leakage scale out of range; bit 1: a load out of range
};

__global__ void __launch_bounds__(256) k_gate_params(GateParamArgs a) {
  __shared__ long long red[256];
  const int64_t gs = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  long long q0 = 0;
  if (gs < a.n_gates) {
    const int32_t c = a.gcell[gs];
    const CellMeta cm = a.meta[c];
    float C = a.net_load[a.gout[gs]];
    if (!(C >= 0.0f && C <= a.load_cap)) {  // keeps every energy inside the fixed-point range
      atomicOr(a.flag, 2);
      C = 0.0f;
    }
    float lam = a.leak_scale ? a.leak_scale[a.gperm[gs]] : 1.0f;
    if (!(lam >= 0.0f && lam <= a.max_scale)) {
      atomicOr(a.flag, 1);
      lam = 0.0f;
    }
    GateParam p;
    p.C = C;
    p.lam = lam;
    a.out[gs] = p;
    const uint32_t s0 = a.ginit[gs] & state_mask(cm.n_in, a.all_pins);
    q0 = (long long)qrate(lam, a.leak[leak_entry_w(a.wide, cm, c, s0)], a.rate_scale);
  }
  red[threadIdx.x] = q0;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) a.l0_part[blockIdx.x] = red[0];
}

// Sum of n partials (one workgroup of 1024 threads) into *out.
__global__ void __launch_bounds__(1024) k_sum_parts(const long long* part, int64_t n, unsigned long long* out) {
  __shared__ long long red[1024];
  long long v = 0;
  for (int64_t i = threadIdx.x; i < n; i += 1024) v += part[i];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = (unsigned long long)red[0];
}

// Leakage rate at every tile start (one workgroup of 1024 threads):
// base[k] = L0 + sum of the tile totals of the steps before tile k, with L0
// the sum of the gate-record kernel's partials.
__global__ void __launch_bounds__(1024) k_tile_base(const long long* l0_part, int64_t n_part, const long long* tot,
                                                    int64_t n_tiles, long long* base) {
  __shared__ long long red[1024];
  __shared__ long long ws[17];
  long long v = 0;
  for (int64_t i = threadIdx.x; i < n_part; i += 1024) v += l0_part[i];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  long long carry = red[0];  // L0
  const int lane = (int)(threadIdx.x & 63), wave = (int)(threadIdx.x >> 6);
  for (int64_t c0 = 0; c0 < n_tiles; c0 += 1024) {
    const int64_t i = c0 + threadIdx.x;
    const long long x = i < n_tiles ? tot[i] : 0;
    long long inc = x;  // inclusive scan within the wavefront
    for (int o = 1; o < 64; o <<= 1) {
      const long long t = __shfl_up(inc, o, 64);
      if (lane >= o) inc += t;
    }
    if (lane == 63) ws[wave] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
      long long acc = 0;
      for (int w = 0; w < 16; ++w) {
        const long long t = ws[w];
        ws[w] = acc;
        acc += t;
      }
      ws[16] = acc;
    }
    __syncthreads();
    if (i < n_tiles) base[i] = carry + ws[wave] + inc - x;
    carry += ws[16];
    __syncthreads();
  }
}

// Power of every bin from the packed forward's per-tile output: X, the
// within-tile exclusive prefix of the leakage steps (exS), the rate at each
// tile start (base) and the tile totals (for the step sum of a partial last
// bin, whose later bins in the tile hold no events).
struct FinTileArgs {
  const int64_t* X;
  const int64_t* exS;
  const long long* base;
  const long long* tot;
  float* P;
  int64_t n_bins, D, t_end;
  int32_t tile_log2;
  double out_scale;     // 2^-m / D
};

__global__ void __launch_bounds__(256) k_finalize_tiles(FinTileArgs a) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= a.n_bins) return;
  const int64_t k = b >> a.tile_log2;
  const int64_t R = (int64_t)a.base[k] + a.exS[b];
  int64_t E;
  if (b == a.n_bins - 1 && a.n_bins * a.D != a.t_end) {
    const int64_t w = a.t_end - b * a.D;
    const int64_t S = (int64_t)a.tot[k] - a.exS[b];
    E = a.X[b] - S * (a.n_bins * a.D - a.t_end) + w * R;
  } else {
    E = a.X[b] + a.D * R;
  }
  a.P[b] = (float)((double)E * a.out_scale);
}

// ---------------------------------------------------------------------------
// forward, one gate per thread (baseline): global int64 atomics per event
// ---------------------------------------------------------------------------
struct SerialArgs {
  EvView ev;
  const GatePrep* gprep;
  LibView lib;
  LutArgs lut;
  BinSpec bins;
  int64_t glitch_clk;   // > 0: glitch detection with this clock period
  unsigned long long* X;
  unsigned long long* S;
};

__global__ void __launch_bounds__(kFwdThreads) k_gate_serial(SerialArgs a) {
  extern __shared__ uint32_t lds[];
  const LdsLib L = stage_library(a.lib, lds);
  __syncthreads();
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= a.ev.n_gates) return;
  const int64_t e0 = a.ev.gate_off[g], e1 = a.ev.gate_off[g + 1];
  if (e1 <= e0) return;
  GateCtx G;
  gate_begin(G, a.gprep, L, g, 0u, a.lut.rate_scale);
  uint32_t par = 0, par_gs = 0;
  int64_t tprev = INT64_MIN;
  const BinSpec& B = a.bins;
  for (int64_t e = e0; e < e1; ++e) {
    const int64_t t = a.ev.t[e];
    const uint32_t b8 = a.ev.pb[e];
    const int pin = (int)(b8 >> 1), v = (int)(b8 & 1u);
    if (t != tprev) {
      par_gs = par;
      tprev = t;
    }
    EventOut o = event_energy(G, L, a.lut, pin, v, a.ev.slew[e], par_gs, par);
    par ^= 1u << (pin & 31);
    if (t < 0 || t >= B.t_end) continue;
    if (a.glitch_clk > 0) {
      const float r = glitch_ratio(a.ev.t, a.ev.pb, a.ev.slew, e0, e, t, pin, a.ev.slew[e], a.glitch_clk);
      o.e = __fmul_rn(o.e, r > 0.f ? r : 1.0f);
    }
    const int64_t b = bin_of(t, B);
    const int64_t rr = t - b * B.D;
    const int64_t x = energy_fixed(o.e, a.lut.two_sh) + (int64_t)o.delta * (B.D - rr);
    atomicAdd(&a.X[b], (unsigned long long)x);
    if (o.delta != 0) atomicAdd(&a.S[b], (unsigned long long)(int64_t)o.delta);
  }
}

// ---------------------------------------------------------------------------
// gate preparation (per call): load interpolation, switching energy, scale
// ---------------------------------------------------------------------------
struct PrepArgs {
  const int32_t* gate_cell;
  const int32_t* gate_out;
  const uint32_t* gate_init;
  const float* net_load;
  const float* leak_scale;   // may be null (all 1)
  const CellMeta* meta;
  const float* leak;
  WideView wide;             // cells with more than 8 state pins
  const float* load;         // [n_cells * n_load]
  const float* load_inv;
  int32_t n_load;
  int64_t n_gates;
  double vdd;
  int32_t sw_mode;
  float rate_scale;   // FP32(2^m * 1e-6)
  float two_sh;       // 2^(m-32)
  float max_scale;
  float load_cap;     // loads must lie in [0, load_cap]
  int32_t all_pins;   // state index over every pin
  GatePrep* out;
  unsigned long long* L0;    // sum of quantised initial leakage rates
  int32_t* flag;             // bit 0: a leakage scale out of range
};

__global__ void __launch_bounds__(256) k_gate_prep(PrepArgs a) {
  __shared__ long long red[256];
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  long long q0 = 0;
  if (g < a.n_gates) {
    const int32_t c = a.gate_cell[g];
    const CellMeta cm = a.meta[c];
    float C = a.net_load[a.gate_out[g]];
    if (!(C >= 0.0f && C <= a.load_cap)) {
      atomicOr(a.flag, 2);
      C = 0.0f;
    }
    float lam = a.leak_scale ? a.leak_scale[g] : 1.0f;
    if (!(lam >= 0.0f && lam <= a.max_scale)) {
      atomicOr(a.flag, 1);
      lam = 0.0f;
    }
    const float* la = a.load + (int64_t)c * a.n_load;
    int j = 0;
    for (int m = 1; m < a.n_load - 1; ++m) j += (la[m] <= C) ? 1 : 0;
    const float inv = a.load_inv[(int64_t)c * a.n_load + j];
    GatePrep p;
    p.cell = c;
    p.init = a.gate_init[g];
    p.jq = j;
    p.beta = __fmul_rn(__fsub_rn(C, la[j]), inv);
    const double v2 = a.vdd * a.vdd;
    if (a.sw_mode == 0) {
      p.esw_rise = (float)(0.5 * (double)C * v2);
      p.esw_fall = p.esw_rise;
    } else {
      p.esw_rise = (float)((double)C * v2);
      p.esw_fall = 0.0f;
    }
    p.lam = lam;
    p.dbeta_dc = inv;
    a.out[g] = p;
    const uint32_t s0 = p.init & state_mask(cm.n_in, a.all_pins);
    q0 = (long long)qrate(lam, a.leak[leak_entry_w(a.wide, cm, c, s0)], a.rate_scale);
  }
  red[threadIdx.x] = q0;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0 && red[0] != 0) atomicAdd(a.L0, (unsigned long long)red[0]);
}

// ---------------------------------------------------------------------------
// finalize: P_b = (X[b] + D * (L0 + sum_{b'<b} S[b'])) * 2^-m / D  (fJ/ps = mW)
// ---------------------------------------------------------------------------
struct FinArgs {
  const int64_t* X;
  const int64_t* S;
  const int64_t* exS;   // exclusive prefix of S
  const unsigned long long* L0;
  float* P;
  int64_t n_bins, D, t_end;
  double out_scale;     // 2^-m / D
};

__global__ void __launch_bounds__(256) k_finalize(FinArgs a) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= a.n_bins) return;
  const int64_t R = (int64_t)*a.L0 + a.exS[b];
  int64_t E;
  if (b == a.n_bins - 1 && a.n_bins * a.D != a.t_end) {
    const int64_t w = a.t_end - b * a.D;
    E = a.X[b] - a.S[b] * (a.n_bins * a.D - a.t_end) + w * R;
  } else {
    E = a.X[b] + a.D * R;
  }
  a.P[b] = (float)((double)E * a.out_scale);
}

// Finalize of concatenated traces. The forward leaves, per bin, the energy X
// and the within-tile exclusive prefix S of the leakage steps, and per tile
// the total of its steps; k_tile_base_batched turns the tile totals of each
// trace into the leakage rate at every tile start (starting from L0 at each
// trace: the traces share the netlist's initial state), and
// k_finalize_batched gives every bin its energy as k_finalize_tiles does.
struct FinTrace {
  int64_t bin_off, n_bins, t_end;
  int64_t tile_off, n_tiles;
  int64_t block_off;   // first finalize block (kFinBins bins each) of the trace
};
constexpr int kFinBins = 256;

__global__ void __launch_bounds__(1024) k_tile_base_batched(const unsigned long long* L0, const FinTrace* traces,
                                                            const long long* tot, long long* base) {
  __shared__ long long ws[17];
  const FinTrace T = traces[blockIdx.x];
  const int lane = (int)(threadIdx.x & 63), wave = (int)(threadIdx.x >> 6);
  long long carry = (long long)*L0;
  for (int64_t c0 = 0; c0 < T.n_tiles; c0 += 1024) {
    const int64_t i = c0 + threadIdx.x;
    const long long x = i < T.n_tiles ? tot[T.tile_off + i] : 0;
    long long inc = x;  // inclusive scan within the wavefront
    for (int o = 1; o < 64; o <<= 1) {
      const long long t = __shfl_up(inc, o, 64);
      if (lane >= o) inc += t;
    }
    if (lane == 63) ws[wave] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
      long long acc = 0;
      for (int w = 0; w < 16; ++w) {
        const long long t = ws[w];
        ws[w] = acc;
        acc += t;
      }
      ws[16] = acc;
    }
    __syncthreads();
    if (i < T.n_tiles) base[T.tile_off + i] = carry + ws[wave] + inc - x;
    carry += ws[16];
    __syncthreads();
  }
}

struct FinBatchArgs {
  const int64_t* X;
  const int64_t* S;            // within-tile exclusive prefix of the steps
  const long long* base;       // rate at every concatenated tile's start
  const long long* tot;        // steps of every concatenated tile
  const FinTrace* traces;
  int32_t n_traces;
  int32_t tile_log2;
  float* P;
  int64_t total_bins, D;
  double out_scale;
};

// One block of kFinBins bins of one trace per workgroup: the trace is found
// once per workgroup (a uniform search, in scalar registers).
__global__ void __launch_bounds__(kFinBins) k_finalize_batched(FinBatchArgs a) {
  const int64_t blk = blockIdx.x;
  int32_t lo = 0, hi = a.n_traces;  // last trace whose blocks start at or before blk
  while (hi - lo > 1) {
    const int32_t mid = (lo + hi) >> 1;
    if (a.traces[mid].block_off <= blk) lo = mid; else hi = mid;
  }
  const FinTrace T = a.traces[lo];
  const int64_t bl = (blk - T.block_off) * kFinBins + threadIdx.x;
  if (bl >= T.n_bins) return;
  const int64_t b = T.bin_off + bl;
  const int64_t k = T.tile_off + (bl >> a.tile_log2);
  const int64_t R = (int64_t)a.base[k] + a.S[b];
  int64_t E;
  if (bl == T.n_bins - 1 && T.n_bins * a.D != T.t_end) {
    const int64_t w = T.t_end - bl * a.D;
    const int64_t S = (int64_t)a.tot[k] - a.S[b];
    E = a.X[b] - S * (T.n_bins * a.D - T.t_end) + w * R;
  } else {
    E = a.X[b] + a.D * R;
  }
  a.P[b] = (float)((double)E * a.out_scale);
}

// ---------------------------------------------------------------------------
// adjoint
// ---------------------------------------------------------------------------
// Per bin: w_b = g_b / D (the density of dL/dP over time) and the suffix
// integral G_b = sum_{b' > b} w_b' * width_b' (width D, the last bin its
// partial width). For a leakage step of size d (nW, unscaled) at time t in
// bin b, d(loss)/d(lambda) gains 1e-6 * d * (w_b * (end_b - t) + G_b), with
// end_b = min((b+1) D, t_end): the integral of w from t to the end of the
// window. Each event adds w_b * dE/dC to its gate's load gradient.
struct AdjArgs {
  EvView ev;
  const uint2* plan;
  const GatePrep* gprep;
  const int32_t* gate_out;
  LibView lib;
  LutArgs lut;
  BinSpec bins;
  const double2* wg;   // [n_bins] (w_b, G_b)
  float dsw_rise, dsw_fall;  // d(switching energy)/dC
  int64_t glitch_clk;  // > 0: glitch detection with this clock period
  double* gC;          // [n_nets]
  double* gL;          // [n_gates] (sum of d * integral, without the 1e-6)
};

struct AdjVisitor {
  const AdjArgs* A;
  const LdsLib* L;
  GateCtx G;
  uint32_t s_cur;
  int64_t g_cur;
  double acc_c, acc_l;
  __device__ __forceinline__ void begin_gate(int64_t g, uint32_t par) {
    gate_begin(G, A->gprep, *L, g, par, A->lut.rate_scale);
    s_cur = (G.gp.init ^ par) & G.in_mask;
    g_cur = g;
    acc_c = 0.0;
    acc_l = 0.0;
  }
  __device__ __forceinline__ void end_gate(int64_t g) {
    if (acc_c != 0.0) unsafeAtomicAdd(&A->gC[A->gate_out[g]], acc_c);
    if (acc_l != 0.0) unsafeAtomicAdd(&A->gL[g], acc_l);
    acc_c = 0.0;
    acc_l = 0.0;
  }
  __device__ __forceinline__ void event(int /*k*/, int64_t e, int64_t t, int pin, int v, float slew, uint32_t par_gs,
                                        uint32_t par) {
    const BinSpec& B = A->bins;
    const uint32_t s_new = (G.gp.init ^ par ^ (1u << (pin & 31))) & G.in_mask;
    if (t < 0 || t >= B.t_end) {  // invalid input: dropped, state still tracked
      if (pin < G.n_state) s_cur = s_new;
      return;
    }
    const int64_t b = bin_of(t, B);
    const double2 wg = A->wg[b];
    const uint32_t s = (G.gp.init ^ par_gs) & G.in_mask;
    const int32_t qb = L->map_q[map_entry(*L, G.cm, G.gp.cell, s, (uint32_t)v)];
    int i;
    float alpha;
    slew_segment(L->slew + G.cm.axis_off, L->slew_inv + G.cm.axis_off, A->lut.n_slew, slew, i, alpha);
    const float4 q = A->lut.quads[qb + i * (A->lut.n_load - 1) + G.gp.jq];
    float dedc = __fmul_rn(bilerp_dbeta(q, alpha), G.gp.dbeta_dc);
    if (pin == G.cm.n_in) dedc = __fadd_rn(dedc, v ? A->dsw_rise : A->dsw_fall);
    if (A->glitch_clk > 0) {
      const float r = glitch_ratio(A->ev.t, A->ev.pb, A->ev.slew, A->ev.gate_off[g_cur], e, t, pin, slew, A->glitch_clk);
      if (r > 0.f) dedc = __fmul_rn(dedc, r);
    }
    acc_c += wg.x * (double)dedc;
    if (pin < G.n_state) {
      const double d = (double)L->leak[leak_entry(*L, G.cm, G.gp.cell, s_new)] -
                       (double)L->leak[leak_entry(*L, G.cm, G.gp.cell, s_cur)];
      const int64_t end_b = min((b + 1) * B.D, B.t_end);
      acc_l += d * (wg.x * (double)(end_b - t) + wg.y);
      s_cur = s_new;
    }
  }
};

__global__ void __launch_bounds__(kFwdThreads) k_adjoint_events(AdjArgs a) {
  extern __shared__ uint32_t lds[];
  const LdsLib L = stage_library(a.lib, lds);
  __syncthreads();
  AdjVisitor vis;
  vis.A = &a;
  vis.L = &L;
  const int64_t kb = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  walk_block(kb, a.ev, a.plan, vis);
}

struct AdjBinArgs {
  const float* gP;
  double* c;       // w_b * width_b
  double* wgtmp;   // w_b
  int64_t n_bins, D, t_end;
};

__global__ void __launch_bounds__(256) k_adj_bins(AdjBinArgs a) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= a.n_bins) return;
  const double w = (double)a.gP[b] / (double)a.D;
  const int64_t width = min((b + 1) * a.D, a.t_end) - b * a.D;
  a.wgtmp[b] = w;
  a.c[b] = w * (double)width;
}

__global__ void __launch_bounds__(256) k_adj_suffix(const double* w, const double* c, const double* exc, double2* wg,
                                                     double* total, int64_t n_bins) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n_bins) return;
  const double tot = exc[n_bins - 1] + c[n_bins - 1];
  wg[b] = make_double2(w[b], tot - (exc[b] + c[b]));
  if (b == 0) *total = tot;
}

struct AdjOutArgs {
  const double* gC;
  const double* gL;
  const double* total;      // integral of w over the window
  const int32_t* gate_cell;
  const uint32_t* gate_init;
  const CellMeta* meta;
  const float* leak;
  WideView wide;             // cells with more than 8 state pins
  float* grad_load;
  float* grad_scale;
  int64_t n_nets, n_gates;
  int32_t all_pins;
};

__global__ void __launch_bounds__(256) k_adj_out(AdjOutArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < a.n_nets) a.grad_load[i] = (float)a.gC[i];
  if (i < a.n_gates) {
    const int32_t c = a.gate_cell[i];
    const CellMeta cm = a.meta[c];
    const uint32_t s0 = a.gate_init[i] & state_mask(cm.n_in, a.all_pins);
    const double base = (double)a.leak[leak_entry_w(a.wide, cm, c, s0)] * *a.total;
    a.grad_scale[i] = (float)(1e-6 * (base + a.gL[i]));
  }
}

// ---------------------------------------------------------------------------
// adjoint, packed layout: one workgroup per (gate block, tile range) item
// ---------------------------------------------------------------------------
// The gates of one gate block accumulate their two gradients in LDS (FP32
// sums over a unit's events, FP64 accumulators per gate); at the end the item
// stores them, with plain coalesced stores, as its own row of a partial
// table, and the output kernel sums a gate's rows in FP64. An item is a run of entries, each one group of the packed layout
// restricted to the lanes (units) of the item's gate block: a group on the
// boundary of two gate blocks appears in both blocks' entries with
// complementary lane ranges. Each event reads its bin's (w_b, G_b) from the
// bin table; one tile's window of it stays in cache while the item walks the
// tile.
struct AdjItem {
  int32_t gb;       // gate block
  int32_t e0, e1;   // entries [e0, e1)
  int32_t q_lo;     // table quads [q_lo, q_lo + q_n) staged in LDS (the block's cell)
  int64_t row;      // first element of the item's row in the partial table (-1: padding, no work)
  int32_t q_n;
  int32_t pad;
};

struct AdjPackedArgs {
  PackedFwdArgs f;            // events, descriptors, gate parameters, library
  const int4* entries;        // (group, tile, first lane, end lane)
  const AdjItem* items;
  const int32_t* gb_start;    // [n_gb + 1] first sorted gate of each gate block
  double2* part;              // partial table: per item and gate (load, leakage)
  int32_t last_w;             // width of the last bin (ps)
  const float2* wg;           // [n_bins] (w_b, Gt_b): Gt_b = integral of w from the end of bin b to the end of its tile
  const double* gtile;        // [n_tiles] integral of w from the end of tile k to the end of the window
  float dsw_rise, dsw_fall;
  int32_t slot_quads;         // LDS table room (quads)
};

// Relaxed FP64 add to LDS (one ds_add_f64).
__device__ __forceinline__ void lds_add_f64(double* p, double v) {
  (void)__hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// One entry's group (loaded into G): per event, the load gradient gains
// w_b * dE/dC and, for an input event, the leakage gradient gains the step of
// the cell leakage times the integral of w from the event to the window end.
// That integral is split at the end of the event's tile: the part inside the
// tile (w_b * (end_b - t) + Gt_b) is summed per event in FP32, the part after
// the tile is the same for every event of the unit, so the unit adds its net
// leakage step times it once, in FP64 (the steps of a gate telescope, so the
// FP32 terms stay as small as the tile's share of the integral). The unit's
// sums go into FP64 LDS accumulators of its gate.
// Lookups are double-buffered by event parity as in the forward.
template <int kS, bool kGl, bool kTabOnly>
__device__ __forceinline__ void adj_process_group(const AdjPackedArgs& a, const LdsLib& L, const GroupRegs<kS>& G,
                                                  bool mine, int32_t tile, int32_t gs0, double* acc_c, double* acc_l,
                                                  const float4* tab, uint32_t q_lo, uint32_t q_n) {
  const BinSpec& B = a.f.bins;
  const uint32_t rmask = (1u << B.r_bits) - 1u;
  const int32_t D32 = (int32_t)B.D;
  const float4* __restrict__ quads = a.f.lut.quads;
  const int len = mine ? G.len : 0;
  const GateParam gp = G.gp;
  const int cell = (int)(G.d.y >> 16);
  const UnitLut u = unit_lut(L, a.f.lut.n_load, cell, gp.C, a.f.v2, a.f.sw_mode);
  const uint32_t jq = u.jq;
  const CellMeta cm = L.meta[cell];
  const float dbdc = len > 0 ? u.dbdc : 0.f;
  const float* lk = L.leak + cm.leak_off;
  const int64_t tile_b0 = (int64_t)tile << B.tile_log2;
  float lk_cur = lk[G.d.y & 0xffffu & state_mask(cm.n_in, L.all_pins)];
  const float lk_first = lk_cur;
  struct Pre {
    float4 q;        // table quad
    float lk_after;  // leakage value of the input state after the event
  };
  auto prefetch = [&](int k, Pre& P) {
    const uint32_t qi = (G.rv[k] & kRowMask) + (uint32_t)jq;
    P.q = kTabOnly ? quad_slot(lds_ptr(tab), q_lo, q_n, qi) : quad_at(quads, lds_ptr(tab), q_lo, q_n, qi);
    P.lk_after = lk[G.wv[k] >> kStateShift];
  };
  // the bins' (w_b, G_b) of all the unit's events, requested together: one
  // cache round trip per group rather than one per event
  float2 wg[kS];
#pragma unroll
  for (int kk = 0; kk < kS; ++kk)
    if (kk < G.kmax && len > kk) wg[kk] = a.wg[tile_b0 + (int64_t)((G.wv[kk] & kTimeMask) >> B.r_bits)];
  float ac = 0.f, al = 0.f;
  Pre pre[2];
  if (len > 0) prefetch(0, pre[0]);
#pragma unroll
  for (int kk = 0; kk < kS; ++kk) {
    if (kk < G.kmax && len > kk) {
      const uint32_t w = G.wv[kk];
      const uint32_t rv = G.rv[kk];
      if (kk + 1 < kS && len > kk + 1) prefetch(kk + 1, pre[(kk + 1) & 1]);
      const Pre& P = pre[kk & 1];
      float dedc = __fmul_rn(bilerp_dbeta(P.q, G.av[kk]), dbdc);
      if (rv & (1u << kOutBit)) dedc = __fadd_rn(dedc, (rv >> 31) ? a.dsw_rise : a.dsw_fall);
      if (kGl) dedc = __fmul_rn(dedc, G.gv[kk]);
      ac = __fmaf_rn(wg[kk].x, dedc, ac);
      // an output event leaves the input state unchanged: step 0, no branch
      const uint32_t tl = w & kTimeMask;
      const int64_t b = tile_b0 + (int64_t)(tl >> B.r_bits);
      const int32_t width = (b == B.n_bins - 1) ? a.last_w : D32;
      const float tail = (float)(width - (int32_t)(tl & rmask));
      al = __fmaf_rn(__fsub_rn(P.lk_after, lk_cur), __fmaf_rn(wg[kk].x, tail, wg[kk].y), al);
      lk_cur = P.lk_after;
    }
  }
  if (len > 0) {
    const int32_t li = (int32_t)(G.d.x & 0x0fffffffu) - gs0;
    const double dl = (double)al + ((double)lk_cur - (double)lk_first) * a.gtile[tile];
    if (ac != 0.f) lds_add_f64(&acc_c[li], (double)ac);
    if (dl != 0.0) lds_add_f64(&acc_l[li], dl);
  }
}

// kTabOnly: every item's LDS table holds all of its cell's quads, so no
// quad comes from global memory and the next group's loads stay in flight
// while a group is processed.
template <int kThreads, int kS, bool kGl, bool kTabOnly>
__global__ void __launch_bounds__(kThreads) k_adjoint_packed(AdjPackedArgs a) {
  extern __shared__ uint32_t lds[];
  const AdjItem it = a.items[blockIdx.x];
  if (it.row < 0) return;  // padding item (the whole workgroup leaves)
  const LdsLib L = stage_library_ml(a.f.lib, lds);
  const int32_t gs0 = a.gb_start[it.gb];
  const int32_t ng = a.gb_start[it.gb + 1] - gs0;
  float4* tab = reinterpret_cast<float4*>(lds + packed_bins_word_offset(a.f.lib.lds_words_ml));
  for (int i = threadIdx.x; i < it.q_n; i += kThreads) tab[i] = a.f.lut.quads[(uint32_t)it.q_lo + (uint32_t)i];
  double* acc_c = reinterpret_cast<double*>(tab + a.slot_quads);
  double* acc_l = acc_c + ng;
  for (int i = threadIdx.x; i < 2 * ng; i += kThreads) acc_c[i] = 0.0;
  const int lane = (int)(threadIdx.x & 63);
  constexpr int nwave = kThreads / 64;
  const int64_t e1 = it.e1;
  // wave-uniform entry index. The entry and group-offset loads are vector
  // loads (through a zero the compiler cannot see through): a scalar load
  // shares its wait counter with LDS, so every LDS access of a group would
  // wait for the next entries' cache round trip.
  int64_t e = it.e0 + (int64_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  int32_t z;
  asm volatile("v_mov_b32 %0, 0" : "=v"(z));
  auto ventry = [&](int64_t i) -> int4 {
    const int4 v = a.entries[i + z];
    return make_int4(__builtin_amdgcn_readfirstlane(v.x), __builtin_amdgcn_readfirstlane(v.y),
                     __builtin_amdgcn_readfirstlane(v.z), __builtin_amdgcn_readfirstlane(v.w));
  };
  auto voff = [&](int32_t g) -> int64_t {
    const int64_t v = a.f.grp_off[(int64_t)g + z];
    return (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(v >> 32)) << 32) |
                     (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int32_t)v));
  };
  GroupRegs<kS> ga, gb;
  bool ma = false, mb = false;
  int32_t ta = 0, tb = 0;
  // loads run ahead of the wavefront's work: the entry two groups ahead, its
  // descriptor and offset one group ahead, the events of the next group
  int4 en2 = make_int4(0, 0, 0, 0);    // entry of group e + 2 nwave
  int4 en1 = make_int4(0, 0, 0, 0);    // entry of group e + nwave
  uint2 dn = make_uint2(0xffffffffu, 0u);
  int64_t offn = 0;
  auto issue = [&](int64_t en, GroupRegs<kS>& R, bool& m, int32_t& t) {
    m = lane >= (en1.z & 0xff) && lane < (en1.z >> 8);
    t = en1.y;
    group_issue<kS, kGl, true>(a.f, dn, offn, R, m);
    en1 = en2;
    if (en + nwave < e1) {
      dn = desc_nt(a.f.desc + (int64_t)en1.x * kGroupUnits + lane);
      offn = voff(en1.x);
    }
    if (en + 2 * nwave < e1) en2 = ventry(en + 2 * nwave);
  };
  if (e < e1) {
    en1 = ventry(e);
    dn = desc_nt(a.f.desc + (int64_t)en1.x * kGroupUnits + lane);
    offn = voff(en1.x);
    if (e + nwave < e1) en2 = ventry(e + nwave);
    issue(e, ga, ma, ta);
  }
  __syncthreads();
  while (e < e1) {
    if (e + nwave < e1) issue(e + nwave, gb, mb, tb);
    adj_process_group<kS, kGl, kTabOnly>(a, L, ga, ma, ta, gs0, acc_c, acc_l, tab, (uint32_t)it.q_lo, (uint32_t)it.q_n);
    e += nwave;
    if (e >= e1) break;
    if (e + nwave < e1) issue(e + nwave, ga, ma, ta);
    adj_process_group<kS, kGl, kTabOnly>(a, L, gb, mb, tb, gs0, acc_c, acc_l, tab, (uint32_t)it.q_lo, (uint32_t)it.q_n);
    e += nwave;
  }
  __syncthreads();
  double2* prow = a.part + it.row;
  for (int i = threadIdx.x; i < ng; i += kThreads) prow[i] = make_double2(acc_c[i], acc_l[i]);
}

// Bin weights of the packed adjoint: (w_b, Gt_b) in FP32 with Gt_b the
// integral of w from the end of bin b to the end of its tile, and per tile
// the integral from the tile's end to the window end (FP64). G_b (the
// integral from the end of bin b to the window end) is Gt_b + gtile[tile].
__global__ void __launch_bounds__(256) k_adj_suffix_tiles(const double* w, const double* c, const double* exc,
                                                          float2* wg, double* gtile, double* total, int64_t n_bins,
                                                          int32_t tile_log2) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n_bins) return;
  const double tot = exc[n_bins - 1] + c[n_bins - 1];
  const int64_t k = b >> tile_log2;
  const int64_t e = min(((k + 1) << tile_log2), n_bins) - 1;   // last bin of the tile
  const double g_end = tot - (exc[e] + c[e]);
  const double g_b = tot - (exc[b] + c[b]);
  wg[b] = make_float2((float)w[b], (float)(g_b - g_end));
  if (b == e) gtile[k] = g_end;
  if (b == 0) *total = tot;
}

// Gradient outputs from the partial table: a sorted gate sums its block's
// rows (one per item of the block) in FP64, adds its load gradient to its
// output net (grad_load zeroed first; a plain store when every net has at most
// one driver) and writes its leakage-scale gradient
// (plus the initial-state leakage times the integral of the bin weights over
// the window).
struct AdjOutSortedArgs {
  const double2* part;
  const int64_t* gb_row;      // [n_gb] first element of the block's rows
  const int32_t* gb_rows;     // [n_gb] rows (items) of the block
  const int32_t* gb_start;    // [n_gb + 1]
  int32_t n_gb;
  const double* total;
  const int32_t* gperm;
  const int32_t* gcell;
  const int32_t* gate_out;
  const uint32_t* gate_init;
  const CellMeta* meta;
  const float* leak;
  WideView wide;             // cells with more than 8 state pins
  float* grad_load;
  float* grad_scale;
  int64_t n_gates;
  int32_t unique_out;         // 1: no net has two drivers (plain stores)
  int32_t all_pins;
};

__global__ void __launch_bounds__(256) k_adj_out_sorted(AdjOutSortedArgs a) {
  const int64_t gs = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gs >= a.n_gates) return;
  int32_t lo = 0, hi = a.n_gb;  // gate block holding gs: gb_start[lo] <= gs < gb_start[hi]
  while (hi - lo > 1) {
    const int32_t mid = (lo + hi) >> 1;
    if (a.gb_start[mid] <= gs) lo = mid; else hi = mid;
  }
  const int64_t ng = a.gb_start[lo + 1] - a.gb_start[lo];
  const double2* p = a.part + a.gb_row[lo] + (gs - a.gb_start[lo]);
  double gc = 0.0, gl = 0.0;
  for (int32_t j = 0; j < a.gb_rows[lo]; ++j) {
    const double2 v = p[j * ng];
    gc += v.x;
    gl += v.y;
  }
  const int32_t g = a.gperm[gs];
  const int32_t c = a.gcell[gs];
  const CellMeta cm = a.meta[c];
  const uint32_t s0 = a.gate_init[g] & state_mask(cm.n_in, a.all_pins);
  a.grad_scale[g] = (float)(1e-6 * ((double)a.leak[leak_entry_w(a.wide, cm, c, s0)] * *a.total + gl));
  if (a.unique_out) {
    a.grad_load[a.gate_out[g]] = (float)gc;
  } else if (gc != 0.0) {
    atomicAdd(&a.grad_load[a.gate_out[g]], (float)gc);
  }
}

// ---------------------------------------------------------------------------
// per-gate report: leakage, internal, switching and glitch energy per gate
// ---------------------------------------------------------------------------
// Gate-major walk (one lane per 16-event block, as the other gate-major
// kernels). Per gate the lane sums, in FP64, the FP32 energies the forward
// uses: internal and switching energy of regular events, the scaled energy of
// glitch events, and the leakage steps d * (t_end - t) (nW ps; the finalize
// kernel adds the initial state's leakage over the window and scales by the
// gate's lambda and 1e-6). A gate entirely inside one lane's block is stored
// with plain stores; the part of a gate that continues into or out of the
// block is added atomically, after the lanes of a wavefront that hold the same
// gate (consecutive lanes) have combined their parts. This is the paper's
// per-gate two-phase reduction (Sec. 4.4) with the first phase in registers.
struct ReportArgs {
  EvView ev;
  const uint2* plan;
  const GatePrep* gprep;
  LibView lib;
  LutArgs lut;
  BinSpec bins;
  int64_t glitch_clk;          // > 0: glitch detection with this clock period
  double* ge;                  // [n_gates * 4]: leak (steps, nW ps), int, sw, gl (fJ); zeroed before
  unsigned long long* t_max;   // latest event time in the window (atomic max; zeroed before)
};

struct RepVisitor {
  const ReportArgs* A;
  const LdsLib* L;
  GateCtx G;
  int64_t e_lo, e_hi;          // the block's events [e_lo, e_hi)
  int64_t g;
  bool spans_in;
  uint32_t s_cur;
  double acc[4];
  int64_t ga = -1, gb = -1;    // gate continuing into / only out of the block
  double va[4], vb[4];
  int64_t tmax = -1;
  __device__ __forceinline__ void begin_gate(int64_t gg, uint32_t par) {
    gate_begin(G, A->gprep, *L, gg, par, A->lut.rate_scale);
    s_cur = (G.gp.init ^ par) & G.in_mask;
    g = gg;
    spans_in = A->ev.gate_off[gg] < e_lo;
    acc[0] = acc[1] = acc[2] = acc[3] = 0.0;
  }
  __device__ __forceinline__ void end_gate(int64_t gg) {
    const bool spans_out = A->ev.gate_off[gg + 1] > e_hi;
    if (!spans_in && !spans_out) {
#pragma unroll
      for (int k = 0; k < 4; ++k) A->ge[4 * gg + k] = acc[k];
    } else if (spans_in) {
      ga = gg;
#pragma unroll
      for (int k = 0; k < 4; ++k) va[k] = acc[k];
    } else {
      gb = gg;
#pragma unroll
      for (int k = 0; k < 4; ++k) vb[k] = acc[k];
    }
    spans_in = false;
  }
  __device__ __forceinline__ void event(int /*k*/, int64_t e, int64_t t, int pin, int v, float slew, uint32_t par_gs,
                                        uint32_t par) {
    const BinSpec& B = A->bins;
    const uint32_t s_new = (G.gp.init ^ par ^ (1u << (pin & 31))) & G.in_mask;
    if (t < 0 || t >= B.t_end) {  // invalid input: dropped, state still tracked
      if (pin < G.n_state) s_cur = s_new;
      return;
    }
    tmax = max(tmax, t);
    const uint32_t s = (G.gp.init ^ par_gs) & G.in_mask;
    const int32_t qb = L->map_q[map_entry(*L, G.cm, G.gp.cell, s, (uint32_t)v)];
    int i;
    float alpha;
    slew_segment(L->slew + G.cm.axis_off, L->slew_inv + G.cm.axis_off, A->lut.n_slew, slew, i, alpha);
    const float4 q = A->lut.quads[qb + i * (A->lut.n_load - 1) + G.gp.jq];
    const float ei = bilerp_quad(q, alpha, G.gp.beta);
    const float es = (pin == G.cm.n_in) ? (v ? G.gp.esw_rise : G.gp.esw_fall) : 0.0f;
    const float r = A->glitch_clk > 0
                        ? glitch_ratio(A->ev.t, A->ev.pb, A->ev.slew, A->ev.gate_off[g], e, t, pin, slew, A->glitch_clk)
                        : -1.0f;
    if (r > 0.f) {
      acc[3] += (double)__fmul_rn(pin == G.cm.n_in ? __fadd_rn(ei, es) : ei, r);
    } else {
      acc[1] += (double)ei;
      acc[2] += (double)es;
    }
    if (pin < G.n_state) {
      acc[0] += ((double)L->leak[leak_entry(*L, G.cm, G.gp.cell, s_new)] -
                 (double)L->leak[leak_entry(*L, G.cm, G.gp.cell, s_cur)]) *
                (double)(B.t_end - t);
      s_cur = s_new;
    }
  }
};

// Sum over consecutive lanes holding the same key (keys do not decrease over
// the lanes that hold one; -1: no value), then the last lane of each run adds
// the sums to the gate's entries.
__device__ __forceinline__ void report_flush(double* ge, int64_t key, double* v) {
  const int lane = (int)(threadIdx.x & 63);
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int64_t ku = __shfl_up(key, o, 64);
    double up[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) up[k] = __shfl_up(v[k], o, 64);
    if (lane >= o && ku == key) {
#pragma unroll
      for (int k = 0; k < 4; ++k) v[k] += up[k];
    }
  }
  const int64_t kd = __shfl_down(key, 1, 64);
  const bool last = (lane == 63) || kd != key;
  if (key >= 0 && last) {
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (v[k] != 0.0) unsafeAtomicAdd(&ge[4 * key + k], v[k]);
  }
}

__global__ void __launch_bounds__(kFwdThreads) k_gate_report(ReportArgs a) {
  extern __shared__ uint32_t lds[];
  const LdsLib L = stage_library(a.lib, lds);
  __syncthreads();
  RepVisitor vis;
  vis.A = &a;
  vis.L = &L;
  const int64_t kb = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  vis.e_lo = kb * kLaneEvents;
  vis.e_hi = min(vis.e_lo + kLaneEvents, a.ev.n);
  vis.spans_in = false;
  walk_block(kb, a.ev, a.plan, vis);
  // every lane of the wavefront takes part in the combines (lanes past the
  // last block hold no value)
  report_flush(a.ge, vis.ga, vis.va);
  report_flush(a.ge, vis.gb, vis.vb);
  int64_t tm = vis.tmax;
  for (int o = 32; o > 0; o >>= 1) tm = max(tm, (int64_t)__shfl_xor(tm, o, 64));
  if ((threadIdx.x & 63) == 0 && tm >= 0) atomicMax(a.t_max, (unsigned long long)tm);
}

// Per gate: leakage energy = lambda * 1e-6 * (leak[s0] * t_end + the summed
// steps), then the design totals (per block, FP64 atomics into tot[4]).
__global__ void __launch_bounds__(256) k_report_finalize(const GatePrep* gprep, const CellMeta* meta,
                                                         const float* leak, WideView wide, int32_t all_pins,
                                                         int64_t n_gates, int64_t t_end, double* ge, double* tot) {
  __shared__ double red[4][256];
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  if (g < n_gates) {
    const GatePrep p = gprep[g];
    const CellMeta cm = meta[p.cell];
    const uint32_t s0 = p.init & state_mask(cm.n_in, all_pins);
    const double el =
        (double)p.lam * 1e-6 * ((double)leak[leak_entry_w(wide, cm, p.cell, s0)] * (double)t_end + ge[4 * g]);
    ge[4 * g] = el;
    v[0] = el;
    v[1] = ge[4 * g + 1];
    v[2] = ge[4 * g + 2];
    v[3] = ge[4 * g + 3];
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) red[k][threadIdx.x] = v[k];
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
#pragma unroll
      for (int k = 0; k < 4; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x < 4) unsafeAtomicAdd(&tot[threadIdx.x], red[threadIdx.x][0]);
}

// Largest bin power (one float per bin; order-preserving integer image of
// the FP32 value for the atomic max).
__device__ __forceinline__ uint32_t float_key(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__global__ void __launch_bounds__(256) k_peak(const float* P, int64_t n, uint32_t* out) {
  uint32_t m = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    m = max(m, float_key(P[i]));
  for (int o = 32; o > 0; o >>= 1) m = max(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0 && m) atomicMax(out, m);
}

// ---------------------------------------------------------------------------
// validation: first offending event in gate-major order
// ---------------------------------------------------------------------------
// Codes ranked by the order the checks are made on one event: time range,
// time order, pin range, pin repeated within a timestamp group, not a toggle.
struct ValArgs {
  EvView ev;
  const uint2* plan;
  const int32_t* gate_cell;
  const uint32_t* gate_init;
  const CellMeta* meta;
  int64_t t_end;
  unsigned long long* first;   // min over (event << 3 | code)
};

struct ValVisitor {
  const ValArgs* A;
  uint32_t init;
  int n_in;
  int64_t gstart;
  unsigned long long best;
  __device__ __forceinline__ void begin_gate(int64_t g, uint32_t) {
    init = A->gate_init[g];
    n_in = A->meta[A->gate_cell[g]].n_in;
    gstart = A->ev.gate_off[g];
  }
  __device__ __forceinline__ void end_gate(int64_t) {}
  __device__ __forceinline__ void event(int /*k*/, int64_t e, int64_t t, int pin, int v, float, uint32_t, uint32_t par) {
    int code = 0;
    if (t < 0 || t >= A->t_end) code = 1;
    else if (e > gstart && A->ev.t[e - 1] > t) code = 2;
    else if (pin > n_in) code = 3;
    else {
      // same pin earlier in this timestamp group (a valid group has at most n_in + 1 events)
      int64_t j = e - 1;
      for (int k = 0; k < 33 && j >= gstart && A->ev.t[j] == t; ++k, --j)
        if ((A->ev.pb[j] >> 1) == pin) { code = 4; break; }
      if (code == 0 && (int)(((init ^ par) >> pin) & 1u) == v) code = 5;
    }
    if (code) {
      const unsigned long long key = ((unsigned long long)e << 3) | (unsigned long long)code;
      if (key < best) best = key;
    }
  }
};

__global__ void __launch_bounds__(kFwdThreads) k_validate(ValArgs a) {
  ValVisitor vis;
  vis.A = &a;
  vis.best = ~0ull;
  const int64_t kb = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  walk_block(kb, a.ev, a.plan, vis);
  if (vis.best != ~0ull) atomicMin(a.first, vis.best);
}

// ---------------------------------------------------------------------------
// streamed windows
// ---------------------------------------------------------------------------
// Times of a window's events made relative to the window start.
__global__ void __launch_bounds__(256) k_shift_times(int64_t* t, int64_t n, int64_t t0) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) t[i] -= t0;
}

// The pin values every gate carries out of a window: each lane block XORs the
// toggles of each gate it holds and applies them to that gate's carried
// values (one atomic per gate and block).
struct CarryVisitor {
  uint32_t* init;
  uint32_t x = 0;
  __device__ __forceinline__ void begin_gate(int64_t, uint32_t) { x = 0; }
  __device__ __forceinline__ void end_gate(int64_t g) {
    if (x) atomicXor(&init[g], x);
  }
  __device__ __forceinline__ void event(int /*k*/, int64_t, int64_t, int pin, int, float, uint32_t, uint32_t) {
    x ^= 1u << (pin & 31);
  }
};

__global__ void __launch_bounds__(kFwdThreads) k_stream_carry(EvView ev, const uint2* plan, uint32_t* init) {
  const int64_t kb = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  CarryVisitor vis;
  vis.init = init;
  walk_block(kb, ev, plan, vis);
}

// per-event trace without the tiled records (one lane block per thread)
struct TraceArgs {
  EvView ev;
  const uint2* plan;
  const GatePrep* gprep;
  LibView lib;
  LutArgs lut;
  BinSpec bins;
  int32_t* state;
  int64_t* bin;
};

struct TraceVisitor {
  const TraceArgs* A;
  const LdsLib* L;
  GateCtx G;
  __device__ __forceinline__ void begin_gate(int64_t g, uint32_t par) {
    gate_begin(G, A->gprep, *L, g, par, A->lut.rate_scale);
  }
  __device__ __forceinline__ void end_gate(int64_t) {}
  __device__ __forceinline__ void event(int /*k*/, int64_t e, int64_t t, int pin, int v, float slew, uint32_t par_gs,
                                        uint32_t par) {
    const EventOut o = event_energy(G, *L, A->lut, pin, v, slew, par_gs, par);
    A->state[e] = o.s;
    A->bin[e] = (t >= 0 && t < A->bins.t_end) ? bin_of(t, A->bins) : -1;
  }
};

__global__ void __launch_bounds__(kFwdThreads) k_event_trace(TraceArgs a) {
  extern __shared__ uint32_t lds[];
  const LdsLib L = stage_library(a.lib, lds);
  __syncthreads();
  TraceVisitor vis;
  vis.A = &a;
  vis.L = &L;
  const int64_t kb = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  walk_block(kb, a.ev, a.plan, vis);
}

// ---------------------------------------------------------------------------
// plan
// ---------------------------------------------------------------------------
// Block b (events [16b, 16b+16)): its first gate, the last gate g with
// gate_off[g] <= 16b. A wavefront's 64 blocks lie in one run of gates, which
// its lanes find together: each round the 64 lanes probe 64 evenly spaced
// gates of the current range and keep the tightest bounds around the run (a
// 65-way search, 3 rounds cut a million gates to a few); each lane then
// bisects the remaining range for its own block.
__global__ void __launch_bounds__(256) k_plan_block_gate(const int64_t* gate_off, int64_t n_gates, int64_t n_events,
                                                         uint2* plan, int64_t n_blocks) {
  const int64_t kb = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = (int)(threadIdx.x & 63);
  const int64_t kw0 = kb - lane;                                        // the wavefront's first block
  const int64_t kw1 = min(kw0 + 64, n_blocks);                          // one past its last block
  if (kw0 >= n_blocks) return;                                          // the whole wavefront
  const int64_t ef = kw0 * kLaneEvents, el = (kw1 - 1) * kLaneEvents;   // first events of its first and last block
  // invariant: gate_off[lo] <= ef and el < gate_off[hi] (gate_off[0] = 0, gate_off[n_gates] = n_events > el)
  int64_t lo = 0, hi = n_gates;
  for (int round = 0; round < 3 && hi - lo > 1; ++round) {
    const int64_t p = lo + (hi - lo) * (lane + 1) / 65;                // lo < p < hi when hi - lo >= 65; else may equal
    const int64_t v = gate_off[p];
    const uint64_t below = __ballot(v <= ef);                           // lanes form a prefix (offsets ascend)
    const uint64_t above = __ballot(v > el);                            // lanes form a suffix
    if (below) lo = __shfl(p, 63 - __clzll((long long)below), 64);
    if (above) hi = __shfl(p, __ffsll((long long)above) - 1, 64);
  }
  if (kb >= n_blocks) return;
  const int64_t e0 = kb * kLaneEvents;
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (gate_off[mid] <= e0) lo = mid; else hi = mid;
  }
  plan[kb] = make_uint2((uint32_t)lo, 0u);
}

// The toggle mask of an event: bit (pin) of its pin_bit byte (pin << 1 | value).
__device__ __forceinline__ uint32_t toggle_bit(uint32_t b) { return 1u << ((b >> 1) & 31u); }
// XOR of the toggle masks of the four events of a 32-bit word of pin_bit bytes.
__device__ __forceinline__ uint32_t toggles4(uint32_t w) {
  return toggle_bit(w & 0xffu) ^ toggle_bit((w >> 8) & 0xffu) ^ toggle_bit((w >> 16) & 0xffu) ^ toggle_bit(w >> 24);
}

// XOR of the toggle masks of a block's events (a whole block is one 16-byte
// load: the caller's arrays are 16-byte aligned).
__global__ void __launch_bounds__(256) k_plan_block_xor(const uint8_t* pb, int64_t n_events, uint32_t* bx,
                                                        int64_t n_blocks) {
  const int64_t kb = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (kb >= n_blocks) return;
  const int64_t e0 = kb * kLaneEvents, e1 = min(e0 + kLaneEvents, n_events);
  uint32_t x = 0;
  if (e1 - e0 == kLaneEvents) {
    const uint4 p4 = *reinterpret_cast<const uint4*>(pb + e0);
    x = toggles4(p4.x) ^ toggles4(p4.y) ^ toggles4(p4.z) ^ toggles4(p4.w);
  } else {
    for (int64_t e = e0; e < e1; ++e) x ^= toggle_bit(pb[e]);
  }
  bx[kb] = x;
}

// Carried parity: with P(x) the XOR of all toggle masks before event x (any
// gate), the parity gate g carries into block b is P(16b) ^ P(gate_off[g]):
// the events of earlier gates cancel. P(gate_off[g]) is the prefix of its
// block plus the block's events before gate_off[g] (that block is whole: it
// ends at or before block b starts).
__global__ void __launch_bounds__(256) k_plan_block_carry(const int64_t* gate_off, const uint8_t* pb,
                                                          const uint32_t* bpre, uint2* plan, int64_t n_blocks) {
  const int64_t kb = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (kb >= n_blocks) return;
  const int64_t e0 = kb * kLaneEvents;
  const uint32_t g = plan[kb].x;
  const int64_t gs = gate_off[g];
  uint32_t carry = 0;
  if (gs < e0) {
    const int64_t kb0 = gs / kLaneEvents;
    const int n = (int)(gs - kb0 * kLaneEvents);   // events of block kb0 before the gate, 0..15
    const uint4 p4 = *reinterpret_cast<const uint4*>(pb + kb0 * kLaneEvents);
    const uint32_t w[4] = {p4.x, p4.y, p4.z, p4.w};
    uint32_t p = bpre[kb0];
#pragma unroll
    for (int i = 0; i < kLaneEvents; ++i)
      if (i < n) p ^= toggle_bit((w[i >> 2] >> (8 * (i & 3))) & 0xffu);
    carry = bpre[kb] ^ p;
  }
  plan[kb].y = carry;
}

// ---------------------------------------------------------------------------
// utilities
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_fill_i32(int32_t* p, int64_t n, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void __launch_bounds__(256) k_fill_u64(unsigned long long* p, int64_t n, unsigned long long v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

}  // namespace gtp
