// kernels.hip — the event kernels: the plain cascade / evaporation pair (the
// paper's Sec. 3 organisation: one cascade per thread, then one de-excitation
// per thread), the persistent work-queue kernel (fused: cascade and
// evaporation as lane states; staged: cascades handed over, then evaporated
// by the same waves once their cascades are over) and the evaporation kernel
// that takes what the staged waves leave.
//
// This file is compiled twice into one library: as is (namespace
// incdev::precise: IEEE division and square root, precise transcendentals)
// and from kernels_fast.hip (namespace incdev::fast: approximate
// transcendentals, reciprocal division, flushed denormals, Sec. 4.2).
#include "kernels.h"

#include <type_traits>

#include "event.h"

#ifndef INC_KERNEL_NS
#define INC_KERNEL_NS precise
#endif

namespace incdev {
namespace INC_KERNEL_NS {

struct KernelArgs {
  const NucTab* nuc;
  int n_targets;
  const XsTab* xs;
  const MassTab* mass;
  BindTab bind;
  EvapTab evap;
  Opts opt;
  size_t n;                  // events in the launch
  const uint8_t* tidx;       // launch inputs (NULL: target 0)
  const float* T0;
  const Segment* segs;       // requests of the launch, sorted by start
  int n_seg;
  uint64_t seed;             // random-stream key of every event of the launch
  unsigned long long* queue; // work-queue heads: [0] events, [1] staged evaporation
  const uint32_t* perm;      // start order: queue position -> launch event (NULL: identity)
  MidState* mid;             // plain kernels: cascade -> evaporation hand-over
  RingDev ring;              // streaming output (rec == NULL: segment arrays)
  int stack_lds;             // stack entries per lane held in LDS
  int chunk;                 // events per work-queue claim
};

__device__ __forceinline__ bool energy_ok(float T0) { return T0 >= 20.0f && T0 <= 250.0f; }

// LDS layout of the event kernels: [n_targets NucTab][NN table][MassTab]
// [writer buffers of the block's waves][LIFO levels: per wave stack_lds x 2 x
// 64 float4].  The NN table is XsLds (columns) or XsPairs (node pairs), see
// xs_lds_bytes.  The evaporation kernels stage only the MassTab (n_targets =
// 0, no NN table: kXsNone), have no stack and larger writer buffers
// (kWriterCapEvap records per wave: nearly every lane emits every step).
__device__ __forceinline__ size_t lds_mass_offset(int n_targets, int xs_layout) {
  return (size_t)n_targets * sizeof(NucTab) + xs_lds_bytes(xs_layout);
}
// First float4 of this lane's column in the LDS stack area (each wave owns
// levels x 2 x 64 consecutive float4).
__device__ __forceinline__ int lds_stack_base(int n_targets, int xs_layout, int levels) {
  return (int)((lds_mass_offset(n_targets, xs_layout) + sizeof(MassTab) +
                (blockDim.x / 64) * (kWriterCap * kRecWords * sizeof(uint32_t))) /
               sizeof(float4)) +
         (int)(threadIdx.x / 64) * levels * 128 + (int)(threadIdx.x % 64);
}
__device__ __forceinline__ void stage_tables(char* lds, const KernelArgs& a, int n_targets, int xs_layout) {
  uint32_t* dst = (uint32_t*)lds;
  const uint32_t* src = (const uint32_t*)a.nuc;
  for (int i = threadIdx.x; i < n_targets * (int)(sizeof(NucTab) / 4); i += blockDim.x) dst[i] = src[i];
  if (xs_layout == kXsColumns) {
    uint32_t* dx = (uint32_t*)(lds + n_targets * sizeof(NucTab));
    const uint32_t* sx = (const uint32_t*)a.xs;
    for (int i = threadIdx.x; i < (int)(sizeof(XsLds) / 4); i += blockDim.x) dx[i] = sx[i];
  } else if (xs_layout == kXsPairs) {
    // the four columns (sigma and majorant of unlike and like pairs) as
    // (v[k], v[k+1]); the last node repeats itself (never read: the table
    // coordinate stays below the last node)
    float2* dx = (float2*)(lds + n_targets * sizeof(NucTab));
    const float* sx = (const float*)a.xs;
    for (int i = threadIdx.x; i < 4 * kXsNodes; i += blockDim.x) {
      const int k = i % kXsNodes;
      dx[i] = make_float2(sx[i], sx[i - k + min(k + 1, kXsNodes - 1)]);
    }
  }
  uint32_t* dm = (uint32_t*)(lds + lds_mass_offset(n_targets, xs_layout));
  const uint32_t* sm = (const uint32_t*)a.mass;
  for (int i = threadIdx.x; i < (int)(sizeof(MassTab) / 4); i += blockDim.x) dm[i] = sm[i];
  __syncthreads();
}

__device__ __forceinline__ void write_residual(inc_residual* r, const Nucleus& nu, float Ex_casc, int nsec, int flags,
                                               int ncoll, int nretry) {
  inc_residual v;
  v.A_f = (uint16_t)max(nu.A, 0);
  v.Z_f = (uint16_t)max(nu.Z, 0);
  v.n_sec = (uint16_t)nsec;
  v.flags = (uint16_t)flags;
  v.Ex_casc = Ex_casc;
  v.Ex_f = nu.E;
  v.p_f[0] = nu.P.x;
  v.p_f[1] = nu.P.y;
  v.p_f[2] = nu.P.z;
  v.n_coll = (uint16_t)min(ncoll, 65535);
  v.n_retry = (uint16_t)min(nretry, 65535);
  *r = v;
}

// Where event i of the launch belongs: its segment, index in the segment.
struct EventRef {
  int seg;
  uint32_t local;
};
__device__ __forceinline__ EventRef event_ref(const KernelArgs& a, size_t i) {
  EventRef e;
  e.seg = a.n_seg == 1 ? 0 : segment_of(a.segs, a.n_seg, (uint32_t)i);
  e.local = (uint32_t)i - a.segs[e.seg].start;
  return e;
}
__device__ __forceinline__ void init_stream(Rng& rng, const KernelArgs& a, EventRef e) {
  rng.init(a.segs[e.seg].first_id + (a.opt.same_stream ? 0 : e.local));
}
__device__ __forceinline__ uint32_t kind_of(uint32_t k, EventRef e) { return k | ((uint32_t)e.seg << 16); }
// Optional history words of an event (inc_output.history): word 0 = uniforms
// drawn from its stream, word 1 = flight segments of its cascade, word 2 =
// the fingerprint of the shells of its tentative collisions.
constexpr int kHistDraws = 0, kHistSegments = 1, kHistShells = 2, kHistWords = 3;
__device__ __forceinline__ void put_hist(const KernelArgs& a, EventRef e, int word, uint32_t v) {
  uint32_t* h = a.segs[e.seg].hist;
  if (h) h[kHistWords * (size_t)e.local + word] = v;
}
// The cascade's words (segments and shell fingerprint) of a finished cascade.
__device__ __forceinline__ void put_hist_cascade(const KernelArgs& a, EventRef e, const Cascade& c) {
  uint32_t* h = a.segs[e.seg].hist;
  if (h) {
    h[kHistWords * (size_t)e.local + kHistSegments] = (uint32_t)c.nseg;
    h[kHistWords * (size_t)e.local + kHistShells] = c.hsh;
  }
}

// Plain cascade kernel: one event per thread (Sec. 3.2).  Each iteration of
// the wave loop advances every live lane by one flight segment together with
// the tentative collision and kinematics it may end in, then the wave writes
// the escaping particles through the compacted writer.
template <bool kRing, bool kHooks>
__global__ void __launch_bounds__(256) k_cascade_plain(KernelArgs a) {
  typename std::conditional<kHooks, Opts, NoHooks>::type op{};
  if constexpr (kHooks) op = a.opt;
  extern __shared__ __align__(16) char lds[];
  stage_tables(lds, a, a.n_targets, kXsColumns);
  const NucTab* snt = (const NucTab*)lds;
  const XsLds& sxs = *(const XsLds*)(lds + a.n_targets * sizeof(NucTab));
  uint32_t* wbuf = (uint32_t*)(lds + lds_mass_offset(a.n_targets, kXsColumns) + sizeof(MassTab)) +
                   (threadIdx.x / 64) * (kWriterCap * kRecWords);
  int fill = 0;

  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool live = i < a.n;
  float T0 = 0.0f;
  int tgt = 0;
  EventRef er = {0, 0};
  Rng rng;
  rng.set_key(a.seed);
  if (live) {
    er = event_ref(a, i);
    T0 = a.T0[i];
    tgt = a.tidx ? (int)a.tidx[i] : 0;
    if (!energy_ok(T0) || tgt >= a.n_targets) {
      MidState m = {};
      m.flags = kFlagRange;
      a.mid[i] = m;
      atomicAdd(&a.segs[er.seg].counters[1], 1ull);
      live = false;
      tgt = 0;
    }
    init_stream(rng, a, er);
  }
  const NucTab& nt = snt[tgt];
  Cascade c;
  cascade_init(c, nt);
  StackEntry stk[kStackDepth];
  c.stk_base = lds_stack_base(a.n_targets, kXsColumns, a.stack_lds);
  c.stk_levels = a.stack_lds;

  while (__any(live)) {
    Emit em;
    em.on = false;
    if (live) {
      int st = flight_step(c, stk, rng, nt, sxs, op, T0, em);
      if (st == kStTent) st = tent_step(c, rng, nt, sxs, op);
      if (st == kStKin) st = kin_step(c, stk, rng, nt, sxs, op);
      if (st == kStDone) {
        const Nucleus r = cascade_residual(c, nt, T0);
        put_hist_cascade(a, er, c);
        MidState m;
        m.A = (int16_t)r.A;
        m.Z = (int16_t)r.Z;
        m.flags = (uint16_t)c.flags;
        m.ncoll = (uint16_t)min(c.ncoll, 65535);
        m.nretry = (uint16_t)min(c.nretry, 65535);
        m.nsec = (uint16_t)(c.nesc0 + c.nesc1);
        m.E = r.E;
        m.P[0] = r.P.x;
        m.P[1] = r.P.y;
        m.P[2] = r.P.z;
        m.drawn = rng.drawn();
        a.mid[i] = m;
        live = false;
      }
    }
    writer_append<kRing>(wbuf, fill, a.segs, a.ring, em.on, er.local, kind_of(em.kind, er), em.T, em.u);
  }
  writer_flush<kRing>(wbuf, fill, a.segs, a.ring);
}

// Plain evaporation kernel: one de-excitation per thread (Sec. 3.3), same
// random stream continued after the cascade's draws.
template <int kExt, bool kRing>
__global__ void __launch_bounds__(256) k_evap_plain(KernelArgs a) {
  extern __shared__ __align__(16) char lds[];
  stage_tables(lds, a, 0, kXsNone);
  const MassTab& smt = *(const MassTab*)lds;
  uint32_t* wbuf = (uint32_t*)(lds + sizeof(MassTab)) + (threadIdx.x / 64) * (kWriterCapEvap * kRecWords);
  int fill = 0;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool live = i < a.n;
  MidState m = {};
  Nucleus nu = {0, 0, 0.0f, {0.0f, 0.0f, 0.0f}};
  Rng rng;
  rng.set_key(a.seed);
  EventRef er = {0, 0};
  int nsec = 0, flags = 0;
  if (live) {
    er = event_ref(a, i);
    inc_residual* res = a.segs[er.seg].res + er.local;
    m = a.mid[i];
    flags = m.flags;
    if (flags & kFlagRange) {
      write_residual(res, nu, 0.0f, 0, flags, 0, 0);
      put_hist(a, er, kHistDraws, 0u);
      put_hist(a, er, kHistSegments, 0u);
      put_hist(a, er, kHistShells, 0u);
      live = false;
    } else {
      nu.A = m.A;
      nu.Z = m.Z;
      nu.E = m.E;
      nu.P = {m.P[0], m.P[1], m.P[2]};
      nsec = m.nsec;
      init_stream(rng, a, er);
      rng.seek(m.drawn);
      if (nu.A <= 0) flags |= kFlagEmpty;
      if (flags) atomicAdd(&a.segs[er.seg].counters[1], 1ull);
      if (nu.A <= 0 || a.opt.no_evaporation) {
        write_residual(res, nu, m.E, nsec, flags, m.ncoll, m.nretry);
        put_hist(a, er, kHistDraws, m.drawn);
        live = false;
      }
    }
  }
  while (__any(live)) {
    Emit em;
    em.on = false;
    if (live) {
      if (evap_step<kExt>(nu, rng, a.bind, a.evap, smt, em)) {
        write_residual(a.segs[er.seg].res + er.local, nu, m.E, nsec, flags, m.ncoll, m.nretry);
        put_hist(a, er, kHistDraws, rng.drawn());
        live = false;
      } else {
        ++nsec;
      }
    }
    writer_append<kRing, kWriterCapEvap>(wbuf, fill, a.segs, a.ring, em.on, er.local, kind_of(em.kind, er), em.T, em.u);
  }
  writer_flush<kRing>(wbuf, fill, a.segs, a.ring);
}

// Persistent kernels.  Every wave keeps 64 events in flight; finished lanes
// refill from a global work queue (one atomic per chunk of 64 events per
// wave; the queue hands out the launch's start order when there is one).
// Each iteration the wave advances the lanes of ONE state (START, FLIGHT,
// TENT, KIN or EVAP), chosen by ballot: a costly state runs once enough lanes
// wait in it (thresholds), else FLIGHT, else whatever state has lanes; once
// no event is left to start, the state with the most lanes.  Lanes in other
// states wait, so every step runs with many lanes together; each lane still
// consumes its own random stream in order, so results do not depend on the
// schedule.
// Sources of evaporation work: chunks of a.chunk consecutive launch events.
// The evaporation kernel takes the chunks listed after the hand-over records
// (mid_bytes): those of waves that took more chunks than they keep.
struct LeftChunks {
  uint32_t* left;
  uint32_t count;
  __device__ __forceinline__ bool claim(unsigned long long& base) {
    uint32_t b = 0;
    if (lane_id() == 0) b = atomicAdd(&left[1], 1u);
    b = (uint32_t)__shfl((int)b, 0);
    if (b >= count) return false;
    base = left[4 + b];
    return true;
  }
};
// A wave's own list: the chunks it took through the cascade, whose hand-over
// records its own lanes wrote.
struct OwnChunks {
  uint32_t list;  // lane i: first event of the wave's i-th chunk
  int count, next;
  __device__ __forceinline__ bool claim(unsigned long long& base) {
    if (next >= count) return false;
    base = (unsigned long long)(uint32_t)__shfl((int)list, next);
    ++next;
    return true;
  }
};

// Evaporation of handed-over events (Sec. 2.4), every lane in the evaporation
// state: a lane whose nucleus has de-excited takes the next event of the
// current chunk, records whose cascade already ended the event (kMidFinal)
// are skipped.  The random stream resumes after the cascade's draws, so the
// results equal the fused kernel's whichever kernel runs this.
template <int kCap, int kExt, bool kRing, class Src>
__device__ __forceinline__ void evap_events(const KernelArgs& a, const MassTab& smt, uint32_t* wbuf, int& fill,
                                            Src& src) {
  unsigned long long chunk_next = 0, chunk_end = 0;
  bool exhausted = false, busy = false;
  EventRef er = {0, 0};
  Rng rng;
  rng.set_key(a.seed);
  Nucleus nu = {0, 0, 0.0f, {0.0f, 0.0f, 0.0f}};
  int nsec = 0, flags = 0, ncoll = 0, nretry = 0;
  float Ex_casc = 0.0f;
  for (;;) {
    const uint64_t need = __ballot(!busy);
    if (need && !exhausted) {
      if (chunk_next == chunk_end) {
        unsigned long long base = 0;
        if (src.claim(base)) {
          chunk_next = base;
          chunk_end = base + a.chunk < a.n ? base + a.chunk : a.n;
        } else {
          exhausted = true;
          chunk_next = chunk_end = 0;
        }
      }
      const unsigned long long avail = chunk_end - chunk_next;
      const uint32_t r = rank_in(need);
      if (!busy && r < avail) {
        const size_t pos = (size_t)(chunk_next + r);
        const size_t ev = a.perm ? (size_t)a.perm[pos] : pos;
        const MidState m = a.mid[ev];
        if (!(m.flags & kMidFinal)) {
          er = event_ref(a, ev);
          nu.A = m.A;
          nu.Z = m.Z;
          nu.E = m.E;
          nu.P = {m.P[0], m.P[1], m.P[2]};
          Ex_casc = m.E;
          nsec = m.nsec;
          flags = m.flags;
          ncoll = m.ncoll;
          nretry = m.nretry;
          init_stream(rng, a, er);
          rng.seek(m.drawn);
          busy = true;
        }
      }
      const unsigned long long cnt = (unsigned long long)__popcll(need);
      chunk_next += cnt < avail ? cnt : avail;
    }
    if (!__any(busy)) {
      if (exhausted) break;
      continue;
    }
    Emit em;
    em.on = false;
    if (busy) {
      if (evap_step<kExt>(nu, rng, a.bind, a.evap, smt, em)) {
        write_residual(a.segs[er.seg].res + er.local, nu, Ex_casc, nsec, flags, ncoll, nretry);
        put_hist(a, er, kHistDraws, rng.drawn());
        if (flags) atomicAdd(&a.segs[er.seg].counters[1], 1ull);
        busy = false;
      } else {
        ++nsec;
      }
    }
    writer_append<kRing, kCap>(wbuf, fill, a.segs, a.ring, em.on, er.local, kind_of(em.kind, er), em.T, em.u);
  }
}

// 4 waves per SIMD (<= 128 VGPRs, 16 per CU): the lane scheduler needs many
// events in flight per CU more than it needs extra registers (measured: 3
// waves per SIMD at 138 VGPRs took 12.3 ms for the 2x10^6-event batch, 4 at
// 128 VGPRs with one VGPR spilled 11.1 ms).
// kFused: the evaporation runs in the same loop as a fifth lane state;
// otherwise (staged mode) the loop hands each finished cascade over and has
// no evaporation state, which leaves it fewer live registers; the wave
// evaporates its hand-overs in a second loop once its cascades are over.
// kPairs: the NN table in LDS as node pairs (XsPairs) instead of columns.
// kExt: the evaporation's optional channels (kExtPhoton, kExtHeavy bits).
template <bool kFused, bool kPairs, int kExt, bool kRing, bool kHooks>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) k_persistent(KernelArgs a) {
  using XS = typename std::conditional<kPairs, XsPairs, XsLds>::type;
  typename std::conditional<kHooks, Opts, NoHooks>::type op{};
  if constexpr (kHooks) op = a.opt;
  constexpr int kLayout = kPairs ? kXsPairs : kXsColumns;
  extern __shared__ __align__(16) char lds[];
  stage_tables(lds, a, a.n_targets, kLayout);
  const NucTab* snt = (const NucTab*)lds;
  const XS& sxs = *(const XS*)(lds + a.n_targets * sizeof(NucTab));
  const MassTab& smt = *(const MassTab*)(lds + lds_mass_offset(a.n_targets, kLayout));
  uint32_t* wbuf = (uint32_t*)(lds + lds_mass_offset(a.n_targets, kLayout) + sizeof(MassTab)) +
                   (threadIdx.x / 64) * (kWriterCap * kRecWords);
  int fill = 0;

  unsigned long long chunk_next = 0, chunk_end = 0;
  bool exhausted = false;
  uint32_t own_list = 0;  // staged: lane i holds the first event of this wave's i-th chunk
  int own_count = 0;
  int st = kStDone;
  EventRef er = {0, 0};
  float T0 = 0.0f;
  int tgt = 0, nsec = 0;
  uint32_t ev_idx = 0;
  float Ex_casc = 0.0f;
  Rng rng;
  rng.set_key(a.seed);
  Cascade c;
  Nucleus nu = {0, 0, 0.0f, {0.0f, 0.0f, 0.0f}};
  StackEntry stk[kStackDepth];
  c.stk_base = lds_stack_base(a.n_targets, kLayout, a.stack_lds);
  c.stk_levels = a.stack_lds;

  for (;;) {
    // ---- refill finished lanes from the work queue
    const uint64_t need = __ballot(st == kStDone);
    if (need && !exhausted) {
      if (chunk_next == chunk_end) {
        unsigned long long base = 0;
        if (lane_id() == 0) base = atomicAdd(a.queue, (unsigned long long)a.chunk);
        base = __shfl(base, 0);
        chunk_next = base;
        chunk_end = base + a.chunk < a.n ? base + a.chunk : a.n;
        if (base >= a.n) {
          exhausted = true;
          chunk_next = chunk_end = a.n;
          // the stragglers of the launch go first from here on
          __builtin_amdgcn_s_setprio(1);
        } else if (!kFused) {
          if (own_count < 64) {
            if (lane_id() == own_count) own_list = (uint32_t)base;
            ++own_count;
          } else {
            // more chunks than the wave keeps: listed for the evaporation kernel
            uint32_t* left = (uint32_t*)(a.mid + a.n);
            if (lane_id() == 0) left[4 + atomicAdd(&left[0], 1u)] = (uint32_t)base;
          }
        }
      }
      const unsigned long long avail = chunk_end - chunk_next;
      const uint32_t r = rank_in(need);
      if (st == kStDone && r < avail) {
        const size_t pos = (size_t)(chunk_next + r);
        const size_t ev = a.perm ? (size_t)a.perm[pos] : pos;
        ev_idx = (uint32_t)ev;
        er = event_ref(a, ev);
        T0 = a.T0[ev];
        tgt = a.tidx ? (int)a.tidx[ev] : 0;
        if (!energy_ok(T0) || tgt >= a.n_targets) {
          tgt = 0;
          const Nucleus z = {0, 0, 0.0f, {0.0f, 0.0f, 0.0f}};
          write_residual(a.segs[er.seg].res + er.local, z, 0.0f, 0, kFlagRange, 0, 0);
          put_hist(a, er, kHistDraws, 0u);
          put_hist(a, er, kHistSegments, 0u);
          put_hist(a, er, kHistShells, 0u);
          atomicAdd(&a.segs[er.seg].counters[1], 1ull);
          if (!kFused) {
            MidState m = {};
            m.flags = kFlagRange | kMidFinal;
            a.mid[ev] = m;
          }
        } else {
          init_stream(rng, a, er);
          cascade_init(c, snt[tgt]);
          nsec = 0;
          st = kStStart;
        }
      }
      const unsigned long long cnt = (unsigned long long)__popcll(need);
      chunk_next += cnt < avail ? cnt : avail;
    }
    if (exhausted && st == kStDone) st = kStIdle;
    const int nF = __popcll(__ballot(st == kStFlight));
    const int nT = __popcll(__ballot(st == kStTent));
    const int nK = __popcll(__ballot(st == kStKin));
    const int nE = kFused ? __popcll(__ballot(st == kStEvap)) : 0;
    const int nS = __popcll(__ballot(st == kStStart));
    if (nF + nT + nK + nE + nS == 0) {
      if (exhausted) break;
      continue;
    }
    // ---- state selection (wave-uniform)
    int run;
    if (exhausted) {
      // no events left to start: the state with the most lanes
      run = kStFlight;
      int best = nF;
      if (nT > best) { run = kStTent; best = nT; }
      if (nK > best) { run = kStKin; best = nK; }
      if (nS > best) { run = kStStart; best = nS; }
      if (nE > best) { run = kStEvap; best = nE; }
    } else if (nK >= a.opt.kin_threshold) run = kStKin;
    else if (nT >= a.opt.tent_threshold) run = kStTent;
    else if (nS >= a.opt.start_threshold) run = kStStart;
    else if (nE >= a.opt.evap_threshold) run = kStEvap;
    else if (nF) run = kStFlight;
    else if (nK) run = kStKin;
    else if (nT) run = kStTent;
    else if (nS) run = kStStart;
    else run = kStEvap;

    Emit em;
    em.on = false;
    if (kFused && run == kStEvap) {
      if (st == kStEvap) {
        if (evap_step<kExt>(nu, rng, a.bind, a.evap, smt, em)) {
          write_residual(a.segs[er.seg].res + er.local, nu, Ex_casc, nsec, c.flags, c.ncoll, c.nretry);
          put_hist(a, er, kHistDraws, rng.drawn());
          if (c.flags) atomicAdd(&a.segs[er.seg].counters[1], 1ull);
          st = kStDone;
        } else {
          ++nsec;
        }
      }
    } else if (st == run) {
      const NucTab& nt = snt[tgt];
      int ns;
      if (run == kStFlight) ns = flight_core(c, stk, nt, em);
      else if (run == kStStart) ns = start_step(c, stk, rng, nt, sxs, op, T0);
      else if (run == kStTent) ns = tent_step(c, rng, nt, sxs, op);
      else ns = kin_step(c, stk, rng, nt, sxs, op);
      if (em.on) ++nsec;
      if (ns == kStDone) {
        nu = cascade_residual(c, nt, T0);
        Ex_casc = nu.E;
        if (nu.A <= 0) c.flags |= kFlagEmpty;
        const bool final = nu.A <= 0 || a.opt.no_evaporation;
        put_hist_cascade(a, er, c);
        if (final) {
          write_residual(a.segs[er.seg].res + er.local, nu, Ex_casc, nsec, c.flags, c.ncoll, c.nretry);
          put_hist(a, er, kHistDraws, rng.drawn());
          if (c.flags) atomicAdd(&a.segs[er.seg].counters[1], 1ull);
        }
        if (!kFused) {
          // staged mode: the evaporation kernel continues this event
          MidState m;
          m.A = (int16_t)nu.A;
          m.Z = (int16_t)nu.Z;
          m.flags = (uint16_t)(c.flags | (final ? kMidFinal : 0));
          m.ncoll = (uint16_t)min(c.ncoll, 65535);
          m.nretry = (uint16_t)min(c.nretry, 65535);
          m.nsec = (uint16_t)nsec;
          m.E = nu.E;
          m.P[0] = nu.P.x;
          m.P[1] = nu.P.y;
          m.P[2] = nu.P.z;
          m.drawn = rng.drawn();
          a.mid[ev_idx] = m;
          st = kStDone;
        } else {
          st = final ? kStDone : kStEvap;
        }
      } else {
        st = ns;
      }
    }
    writer_append<kRing>(wbuf, fill, a.segs, a.ring, em.on, er.local, kind_of(em.kind, er), em.T, em.u);
  }
  if (!kFused) {
    // Staged mode: this wave's cascades are over and no event is left to
    // start.  While other waves finish their longest cascades, evaporate the
    // events this wave handed over (its own lanes wrote those records, so
    // only wave-level ordering is needed), at the lowest priority; the
    // evaporation kernel that follows takes whatever is left.
    __builtin_amdgcn_s_setprio(0);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    OwnChunks src = {own_list, own_count, 0};
    evap_events<kWriterCap, kExt, kRing>(a, smt, wbuf, fill, src);
  }
  writer_flush<kRing>(wbuf, fill, a.segs, a.ring);
}

// Staged mode, second kernel: the evaporation of the handed-over events the
// cascade kernel's waves did not evaporate themselves (the chunks listed
// after the hand-over records), as a persistent work-queue kernel.
template <int kExt, bool kRing>
__global__ void __launch_bounds__(256) k_evap_persistent(KernelArgs a) {
  // usually nothing is left: the cascade waves evaporated what they handed over
  uint32_t* left = (uint32_t*)(a.mid + a.n);
  const uint32_t count = __hip_atomic_load(&left[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (count == 0) return;
  extern __shared__ __align__(16) char lds[];
  stage_tables(lds, a, 0, kXsNone);
  const MassTab& smt = *(const MassTab*)lds;
  uint32_t* wbuf = (uint32_t*)(lds + sizeof(MassTab)) + (threadIdx.x / 64) * (kWriterCapEvap * kRecWords);
  int fill = 0;
  LeftChunks src = {left, count};
  evap_events<kWriterCapEvap, kExt, kRing>(a, smt, wbuf, fill, src);
  writer_flush<kRing>(wbuf, fill, a.segs, a.ring);
}

// Evaporation alone (Sec. 2.4) of given excited nuclei: each nucleus becomes a
// hand-over record with no draws consumed, so it evaporates on its event's
// stream from the first draw, and every chunk of the launch is listed for the
// evaporation kernel.  A nucleus outside the tables' (A, Z) range, with an
// excitation outside [0, kMaxExcitation] or a non-finite momentum is final
// at once, flagged out of range.
__global__ void k_excited_setup(KernelArgs a, ExcitedDesc x) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t* left = (uint32_t*)(a.mid + a.n);
  if (i == 0) {
    left[0] = (uint32_t)((a.n + a.chunk - 1) / a.chunk);
    left[1] = 0u;
  }
  if (i >= a.n) return;
  if (i % a.chunk == 0) left[4 + i / a.chunk] = (uint32_t)i;
  const int A = x.A[i], Z = x.Z[i];
  const float E = x.Ex[i];
  float P[3] = {0.0f, 0.0f, 0.0f};
  if (x.P) {
    P[0] = x.P[3 * i];
    P[1] = x.P[3 * i + 1];
    P[2] = x.P[3 * i + 2];
  }
  const bool ok = A >= 1 && A <= a.bind.amax && Z <= A && Z <= a.bind.zmax && E >= 0.0f && E <= kMaxExcitation &&
                  isfinite(P[0]) && isfinite(P[1]) && isfinite(P[2]);
  MidState m = {};
  const EventRef er = event_ref(a, i);
  put_hist(a, er, kHistSegments, 0u);
  put_hist(a, er, kHistShells, 0u);
  if (ok) {
    m.A = (int16_t)A;
    m.Z = (int16_t)Z;
    m.E = E;
    m.P[0] = P[0];
    m.P[1] = P[1];
    m.P[2] = P[2];
  } else {
    m.flags = kFlagRange | kMidFinal;
    const Nucleus z = {0, 0, 0.0f, {0.0f, 0.0f, 0.0f}};
    write_residual(a.segs[er.seg].res + er.local, z, 0.0f, 0, kFlagRange, 0, 0);
    put_hist(a, er, kHistDraws, 0u);
    atomicAdd(&a.segs[er.seg].counters[1], 1ull);
  }
  a.mid[i] = m;
}

// Zero the segments' counters, the work-queue heads and (staged) the list of
// chunks left to the evaporation kernel (a fill kernel rather than a memset,
// so the launch sequence stays capturable in a graph).
__global__ void k_zero_counters(const Segment* segs, int n_seg, unsigned long long* queue, uint32_t* left) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_seg) {
    segs[i].counters[0] = 0ull;
    segs[i].counters[1] = 0ull;
  }
  if (i == 0) {
    queue[0] = 0ull;
    queue[1] = 0ull;
    if (left) left[0] = left[1] = 0u;
  }
}

// ================================================================== vertex
// Event-based pipeline (the restructuring Sec. 4.2 suggests: separate kernels
// for the vertex types, over compacted queues), kept as a measured rival of
// the persistent kernel.  A window of W in-flight events keeps its state in
// device memory (VSlot, with a LIFO of kStackDepth entries per slot); one
// kernel per vertex type runs the events that stand at that vertex, every
// lane busy with one of them.  One cycle runs kVPairs pairs of stages FLIGHT
// (flight segments until a tentative collision or the end of the cascade; an
// escape or a transparent pass starts the next flight at once) and TENT
// (tentative collisions; a null collision goes on in the next FLIGHT stage),
// then KIN (accepted or blocked collisions), EVAP (the whole evaporation of a
// finished cascade), REFILL (slots whose event ended take the next events of
// the launch, in start order, and enter them) and SWAP.  A slot handed to a
// vertex type joins the queue of the next stage of that type in the cycle, or
// of its first stage in the next cycle.  Each event runs the same steps on its
// own stream as in the other modes, so the results are the same.
enum { kVFlight = 0, kVTent = 1, kVKin = 2, kVEvap = 3, kVFree = 4, kVTypes = 5 };
constexpr int kVPairs = 3;
constexpr int kVStages = 2 * kVPairs + 3;
constexpr int kVRefill = kVStages - 1;
__host__ __device__ constexpr int vstage_type(int k) {
  return k < 2 * kVPairs ? (k & 1) : (k == 2 * kVPairs ? kVKin : (k == 2 * kVPairs + 1 ? kVEvap : kVFree));
}
// Destination stage of a slot handed to type t by stage k: bit 8 set for the
// next cycle.
__host__ __device__ constexpr int vdest(int k, int t) {
  for (int j = k + 1; j < kVStages; ++j)
    if (vstage_type(j) == t) return j;
  for (int j = 0; j < kVStages; ++j)
    if (vstage_type(j) == t) return j | 256;
  return 0;
}
static_assert(vdest(kVRefill, kVFlight) == 256 && vdest(1, kVFlight) == 2 && vdest(2 * kVPairs - 1, kVFlight) == 256,
              "stage order");

struct __align__(16) VSlot {
  Cascade c;
  Rng rng;
  Nucleus nu;
  EventRef er;
  float T0, Ex_casc;
  int tgt, nsec;
};

struct VertexArgs {
  VSlot* slots;
  StackEntry* stacks;  // kStackDepth per slot
  uint32_t* queues;    // [2 parities][kVStages][window]
  uint32_t* ctl;       // [0] parity of this cycle, [1] slots holding an event, [2] done, [4 + 16 p + k] counts
  uint32_t window;
};
static_assert(4 + 16 + kVStages <= kVertexCtlWords && kVStages <= 16, "control words");

__device__ __forceinline__ uint32_t* vq(const VertexArgs& v, int p, int k) {
  return v.queues + ((size_t)p * kVStages + k) * v.window;
}
__device__ __forceinline__ uint32_t* vcnt(const VertexArgs& v, int p, int k) { return v.ctl + 4 + 16 * p + k; }

// Hand `slot` to type t (lanes with `on`; every lane of the wave calls) from
// stage kFrom.  One atomic per wave and destination queue.
template <int kFrom>
__device__ __forceinline__ void vpush(const VertexArgs& v, bool on, int t, int cur, uint32_t slot) {
#pragma unroll
  for (int q = 0; q < kVTypes; ++q) {
    const uint64_t m = __ballot(on && t == q);
    if (!m) continue;
    constexpr int kD[kVTypes] = {vdest(kFrom, 0), vdest(kFrom, 1), vdest(kFrom, 2), vdest(kFrom, 3), vdest(kFrom, 4)};
    const int p = (kD[q] & 256) ? 1 - cur : cur;
    const int k = kD[q] & 255;
    const int leader = __ffsll((unsigned long long)m) - 1;
    uint32_t base = 0;
    if (lane_id() == leader) base = atomicAdd(vcnt(v, p, k), (uint32_t)__popcll(m));
    base = (uint32_t)__shfl((int)base, leader);
    if (on && t == q) vq(v, p, k)[base + rank_in(m)] = slot;
  }
}

// A slot's state to and from separate locals (as the persistent kernel keeps
// them), so that every field can stay in registers.
__device__ __forceinline__ void vload(const VSlot& g, Cascade& c, Rng& rng, Nucleus& nu, EventRef& er, float& T0,
                                      float& Ex_casc, int& tgt, int& nsec) {
  c = g.c;
  rng = g.rng;
  nu = g.nu;
  er = g.er;
  T0 = g.T0;
  Ex_casc = g.Ex_casc;
  tgt = g.tgt;
  nsec = g.nsec;
}
__device__ __forceinline__ void vstore(VSlot& g, const Cascade& c, const Rng& rng, const Nucleus& nu, EventRef er,
                                       float T0, float Ex_casc, int tgt, int nsec) {
  g.c = c;
  g.rng = rng;
  g.nu = nu;
  g.er = er;
  g.T0 = T0;
  g.Ex_casc = Ex_casc;
  g.tgt = tgt;
  g.nsec = nsec;
}

// End of a cascade, as in the fused persistent kernel: the residual nucleus;
// a final one (empty, or evaporation off) is written out and frees its slot.
__device__ __forceinline__ int vtx_cascade_end(const KernelArgs& a, Cascade& c, const Rng& rng, Nucleus& nu,
                                               EventRef er, float T0, float& Ex_casc, int nsec, const NucTab& nt) {
  nu = cascade_residual(c, nt, T0);
  Ex_casc = nu.E;
  if (nu.A <= 0) c.flags |= kFlagEmpty;
  put_hist_cascade(a, er, c);
  if (nu.A <= 0 || a.opt.no_evaporation) {
    write_residual(a.segs[er.seg].res + er.local, nu, Ex_casc, nsec, c.flags, c.ncoll, c.nretry);
    put_hist(a, er, kHistDraws, rng.drawn());
    if (c.flags) atomicAdd(&a.segs[er.seg].counters[1], 1ull);
    return kVFree;
  }
  return kVEvap;
}

__global__ void k_vertex_init(VertexArgs v, uint32_t w) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < w) vq(v, 0, kVRefill)[i] = i;
  if (i < kVertexCtlWords) v.ctl[i] = 0u;
  __syncthreads();  // (block 0 only writes ctl)
  if (i == 0) {
    v.ctl[1] = w;
    *vcnt(v, 0, kVRefill) = w;
  }
}

// One stage (FLIGHT, TENT, KIN or EVAP) over this cycle's queue of the stage,
// grid-stride.
template <int kStage, int kExt>
__global__ void __launch_bounds__(256) k_vertex(KernelArgs a, VertexArgs v) {
  constexpr int kType = vstage_type(kStage);
  const int cur = (int)v.ctl[0];
  const uint32_t n = *vcnt(v, cur, kStage);
  if ((uint32_t)(blockIdx.x * blockDim.x) >= n) return;
  constexpr bool kEvap = kType == kVEvap;
  constexpr int kLayout = kEvap ? kXsNone : kXsColumns;
  extern __shared__ __align__(16) char lds[];
  const int ntab = kEvap ? 0 : a.n_targets;
  stage_tables(lds, a, ntab, kLayout);
  const NucTab* snt = (const NucTab*)lds;
  const XsLds& sxs = *(const XsLds*)(lds + ntab * sizeof(NucTab));
  const MassTab& smt = *(const MassTab*)(lds + lds_mass_offset(ntab, kLayout));
  constexpr int kCap = kEvap ? kWriterCapEvap : kWriterCap;
  uint32_t* wbuf = (uint32_t*)(lds + lds_mass_offset(ntab, kLayout) + sizeof(MassTab)) +
                   (threadIdx.x / 64) * (kCap * kRecWords);
  int fill = 0;
  for (uint32_t base = blockIdx.x * blockDim.x; base < n; base += gridDim.x * blockDim.x) {
    const uint32_t i = base + threadIdx.x;
    const bool live = i < n;
    const uint32_t slot = live ? vq(v, cur, kStage)[i] : 0u;
    Cascade c;
    Rng rng;
    Nucleus nu;
    EventRef er;
    float T0, Ex_casc;
    int tgt, nsec;
    // (slot 0 for idle lanes: read, never written)
    vload(v.slots[slot], c, rng, nu, er, T0, Ex_casc, tgt, nsec);
    StackEntry* stk = v.stacks + (size_t)slot * kStackDepth;
    int next = kVFree;
    if constexpr (kEvap) {
      bool act = live;
      while (__any(act)) {
        Emit em;
        em.on = false;
        if (act) {
          if (evap_step<kExt>(nu, rng, a.bind, a.evap, smt, em)) {
            write_residual(a.segs[er.seg].res + er.local, nu, Ex_casc, nsec, c.flags, c.ncoll, c.nretry);
            put_hist(a, er, kHistDraws, rng.drawn());
            if (c.flags) atomicAdd(&a.segs[er.seg].counters[1], 1ull);
            act = false;
          } else {
            ++nsec;
          }
        }
        writer_append<false, kCap>(wbuf, fill, a.segs, a.ring, em.on, er.local, kind_of(em.kind, er), em.T, em.u);
      }
    } else {
      const NucTab& nt = snt[live ? tgt : 0];
      if constexpr (kType == kVFlight) {
        bool act = live;
        while (__any(act)) {
          Emit em;
          em.on = false;
          if (act) {
            int ns = flight_core(c, stk, nt, em);
            if (em.on) ++nsec;
            if (ns == kStStart) ns = start_step(c, stk, rng, nt, sxs, a.opt, T0);
            if (ns == kStTent) {
              next = kVTent;
              act = false;
            } else if (ns == kStDone) {
              next = vtx_cascade_end(a, c, rng, nu, er, T0, Ex_casc, nsec, nt);
              act = false;
            }
          }
          writer_append<false>(wbuf, fill, a.segs, a.ring, em.on, er.local, kind_of(em.kind, er), em.T, em.u);
        }
      } else if constexpr (kType == kVTent) {
        if (live) next = tent_step(c, rng, nt, sxs, a.opt) == kStKin ? kVKin : kVFlight;
      } else {
        if (live) {
          const int ns = kin_step(c, stk, rng, nt, sxs, a.opt);
          next = ns == kStDone ? vtx_cascade_end(a, c, rng, nu, er, T0, Ex_casc, nsec, nt) : kVFlight;
        }
      }
    }
    if (live && next != kVFree) vstore(v.slots[slot], c, rng, nu, er, T0, Ex_casc, tgt, nsec);
    vpush<kStage>(v, live, next, cur, slot);
  }
  writer_flush<false>(wbuf, fill, a.segs, a.ring);
}

// REFILL: every freed slot takes the next event of the launch (in start
// order; out-of-range inputs are written out flagged and skipped) and enters
// the nucleus; a slot that finds none is retired.  Grid-stride.
__global__ void __launch_bounds__(256) k_vertex_refill(KernelArgs a, VertexArgs v) {
  const int cur = (int)v.ctl[0];
  const uint32_t n = *vcnt(v, cur, kVRefill);
  if ((uint32_t)(blockIdx.x * blockDim.x) >= n) return;
  extern __shared__ __align__(16) char lds[];
  stage_tables(lds, a, a.n_targets, kXsColumns);
  const NucTab* snt = (const NucTab*)lds;
  const XsLds& sxs = *(const XsLds*)(lds + a.n_targets * sizeof(NucTab));
  for (uint32_t base = blockIdx.x * blockDim.x; base < n; base += gridDim.x * blockDim.x) {
    const uint32_t i = base + threadIdx.x;
    const bool live = i < n;
    const uint32_t slot = live ? vq(v, cur, kVRefill)[i] : 0u;
    EventRef er = {0, 0};
    float T0 = 0.0f;
    int tgt = 0;
    bool need = live, got = false;
    while (__any(need)) {
      const uint64_t m = __ballot(need);
      const int leader = __ffsll((unsigned long long)m) - 1;
      unsigned long long first = 0;
      if (lane_id() == leader) first = atomicAdd(a.queue, (unsigned long long)__popcll(m));
      first = __shfl(first, leader);
      if (need) {
        const unsigned long long pos = first + rank_in(m);
        if (pos >= a.n) {
          need = false;
        } else {
          const size_t ev = a.perm ? (size_t)a.perm[pos] : (size_t)pos;
          er = event_ref(a, ev);
          T0 = a.T0[ev];
          tgt = a.tidx ? (int)a.tidx[ev] : 0;
          if (!energy_ok(T0) || tgt >= a.n_targets) {
            tgt = 0;
            const Nucleus z = {0, 0, 0.0f, {0.0f, 0.0f, 0.0f}};
            write_residual(a.segs[er.seg].res + er.local, z, 0.0f, 0, kFlagRange, 0, 0);
            put_hist(a, er, kHistDraws, 0u);
            put_hist(a, er, kHistSegments, 0u);
            put_hist(a, er, kHistShells, 0u);
            atomicAdd(&a.segs[er.seg].counters[1], 1ull);
          } else {
            need = false;
            got = true;
          }
        }
      }
    }
    if (got) {
      StackEntry* stk = v.stacks + (size_t)slot * kStackDepth;
      Rng rng;
      rng.set_key(a.seed);
      init_stream(rng, a, er);
      const NucTab& nt = snt[tgt];
      Cascade c;
      cascade_init(c, nt);
      c.stk_base = 0;
      c.stk_levels = 0;  // the whole LIFO in the slot's device memory
      (void)start_step(c, stk, rng, nt, sxs, a.opt, T0);  // the entry: always a flight
      const Nucleus nu = {0, 0, 0.0f, {0.0f, 0.0f, 0.0f}};
      vstore(v.slots[slot], c, rng, nu, er, T0, 0.0f, tgt, 0);
    }
    vpush<kVRefill>(v, got, kVFlight, cur, slot);
    const uint64_t retired = __ballot(live && !got);
    if (retired && lane_id() == __ffsll((unsigned long long)retired) - 1)
      atomicSub(&v.ctl[1], (uint32_t)__popcll(retired));
  }
}

// SWAP: this cycle's queues are spent; the next cycle's become current.
__global__ void k_vertex_swap(VertexArgs v) {
  if (threadIdx.x != 0) return;
  const int cur = (int)v.ctl[0];
  for (int k = 0; k < kVStages; ++k) *vcnt(v, cur, k) = 0u;
  v.ctl[0] = (uint32_t)(1 - cur);
  v.ctl[2] = v.ctl[1] == 0u ? 1u : 0u;
}

// ================================================================ launchers
size_t lds_bytes(int n_targets, int block, int xs_layout, int stack_levels) {
  const bool events = xs_layout != kXsNone;
  return (size_t)n_targets * sizeof(NucTab) + xs_lds_bytes(xs_layout) + sizeof(MassTab) +
         (size_t)(block / 64) * (events ? kWriterCap : kWriterCapEvap) * kRecWords * sizeof(uint32_t) +
         (size_t)stack_levels * 2 * block * sizeof(float4);
}

int stack_levels(int mode, int n_targets, int block, int waves_per_cu, int xs_layout) {
  int dev = 0, lds_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) != hipSuccess ||
      lds_cu <= 0)
    return 0;
  if (mode == INC_MODE_PLAIN) xs_layout = kXsColumns;
  const size_t base = lds_bytes(n_targets, block, xs_layout, 0);
  int occ = 0;
  const bool pairs = xs_layout == kXsPairs;
  const void* fn = mode == INC_MODE_PLAIN        ? (const void*)k_cascade_plain<false, false>
                   : mode == INC_MODE_PERSISTENT ? (pairs ? (const void*)k_persistent<true, true, 0, false, false>
                                                          : (const void*)k_persistent<true, false, 0, false, false>)
                                                 : (pairs ? (const void*)k_persistent<false, true, 0, false, false>
                                                          : (const void*)k_persistent<false, false, 0, false, false>);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fn, block, base) != hipSuccess || occ < 1) return 0;
  int blocks = occ;
  if (mode != INC_MODE_PLAIN) {
    const int want = (waves_per_cu * 64 + block - 1) / block;
    if (want < blocks) blocks = want < 1 ? 1 : want;
  }
  // keep a 1 KiB allocation margin per workgroup
  const size_t budget = (size_t)lds_cu / blocks;
  if (budget < base + 1024) return 0;
  const size_t levels = (budget - base - 1024) / (2 * (size_t)block * sizeof(float4));
  return levels > (size_t)kStackLdsMax ? kStackLdsMax : (int)levels;
}

int evap_blocks_per_cu(int block) {
  int occ = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void*)k_evap_persistent<0, false>, block,
                                                   lds_bytes(0, block, kXsNone, 0)) != hipSuccess ||
      occ < 1)
    return 1;
  return occ;
}

static KernelArgs kernel_args(const LaunchDesc& L) {
  KernelArgs a;
  a.nuc = L.nuc;
  a.n_targets = L.n_targets;
  a.xs = L.xs;
  a.mass = L.mass;
  a.bind = {L.bind, L.zmax + 1, L.amax, L.zmax, L.chan, L.heavy_rows, L.heavy_mass};
  a.evap = L.evap;
  a.opt.no_pauli = L.opt.no_pauli;
  a.opt.no_evaporation = L.opt.no_evaporation;
  a.opt.stop_after_first = L.opt.stop_after_first;
  a.opt.const_sigma_mb = L.opt.const_sigma_mb;
  a.opt.fixed_b = L.fixed_b_set ? L.opt.fixed_b : -1.0f;
  a.opt.evap_threshold = L.evap_threshold;
  a.opt.tent_threshold = L.tent_threshold;
  a.opt.kin_threshold = L.kin_threshold;
  a.opt.start_threshold = L.start_threshold;
  a.opt.same_stream = L.opt.same_stream;
  a.n = L.n;
  a.tidx = L.tidx;
  a.T0 = L.T0;
  a.segs = L.segs;
  a.n_seg = L.n_seg;
  a.seed = L.seed;
  a.queue = L.queue;
  a.perm = L.perm;
  a.mid = L.mid;
  a.ring = L.ring;
  a.stack_lds = L.stack_lds;
  a.chunk = L.chunk > 0 ? L.chunk : kChunkEvents;
  return a;
}

// The kernels of the default model without test hooks carry neither the
// hooks (kHooks) nor the ring (kRing); a context with hooks set, or a ring
// launch, takes the instances with the runtime hooks.  The evaporation
// options' instantiations (kExt != 0), the hooks' and the ring's take the
// columns layout.
template <int kExt, bool kRing, bool kHooks>
static void launch_ext(const LaunchDesc& L, const KernelArgs& a, hipStream_t s) {
  const int block = L.block;
  if (L.mode == INC_MODE_PLAIN) {
    const unsigned grid = (unsigned)((L.n + block - 1) / block);
    hipLaunchKernelGGL((k_cascade_plain<kRing, kHooks>), dim3(grid), dim3(block),
                       lds_bytes(L.n_targets, block, kXsColumns, L.stack_lds), s, a);
    hipLaunchKernelGGL((k_evap_plain<kExt, kRing>), dim3(grid), dim3(block), lds_bytes(0, block, kXsNone, 0), s, a);
    return;
  }
  constexpr bool kCols = kExt != 0 || kRing || kHooks;
  const dim3 grid(L.persistent_blocks);
  const size_t lds = lds_bytes(L.n_targets, block, L.xs_pairs && !kCols ? kXsPairs : kXsColumns, L.stack_lds);
  if (L.mode == INC_MODE_STAGED) {
    if (!kCols && L.xs_pairs)
      hipLaunchKernelGGL((k_persistent<false, true, 0, false, false>), grid, dim3(block), lds, s, a);
    else
      hipLaunchKernelGGL((k_persistent<false, false, kExt, kRing, kHooks>), grid, dim3(block), lds, s, a);
    hipLaunchKernelGGL((k_evap_persistent<kExt, kRing>), dim3(L.evap_blocks), dim3(block),
                       lds_bytes(0, block, kXsNone, 0), s, a);
  } else {
    if (!kCols && L.xs_pairs)
      hipLaunchKernelGGL((k_persistent<true, true, 0, false, false>), grid, dim3(block), lds, s, a);
    else
      hipLaunchKernelGGL((k_persistent<true, false, kExt, kRing, kHooks>), grid, dim3(block), lds, s, a);
  }
}

template <int kExt>
static void launch_ext_out(const LaunchDesc& L, const KernelArgs& a, hipStream_t s) {
  const bool ring = L.ring.tag || L.ring.done;
  const bool hooks = L.opt.no_pauli || L.opt.stop_after_first || L.opt.const_sigma_mb > 0.0f || L.fixed_b_set;
  if (ring) launch_ext<kExt, true, true>(L, a, s);
  else if (hooks) launch_ext<kExt, false, true>(L, a, s);
  else launch_ext<kExt, false, false>(L, a, s);
}

static int ext_of(const LaunchDesc& L) { return (L.photon ? kExtPhoton : 0) | (L.heavy ? kExtHeavy : 0); }

hipError_t launch_events(const LaunchDesc& L, hipStream_t s) {
  const KernelArgs a = kernel_args(L);
  hipLaunchKernelGGL(k_zero_counters, dim3((L.n_seg + 63) / 64), dim3(64), 0, s, L.segs, L.n_seg, L.queue,
                     L.mode == INC_MODE_STAGED ? (uint32_t*)(L.mid + L.n) : nullptr);
  switch (ext_of(L)) {
    case 0: launch_ext_out<0>(L, a, s); break;
    case kExtPhoton: launch_ext_out<kExtPhoton>(L, a, s); break;
    case kExtHeavy: launch_ext_out<kExtHeavy>(L, a, s); break;
    default: launch_ext_out<kExtPhoton | kExtHeavy>(L, a, s); break;
  }
  return hipGetLastError();
}

hipError_t launch_evaporation(const LaunchDesc& L, const ExcitedDesc& x, hipStream_t s) {
  const KernelArgs a = kernel_args(L);
  hipLaunchKernelGGL(k_zero_counters, dim3((L.n_seg + 63) / 64), dim3(64), 0, s, L.segs, L.n_seg, L.queue,
                     (uint32_t*)nullptr);
  hipLaunchKernelGGL(k_excited_setup, dim3((unsigned)((L.n + 255) / 256)), dim3(256), 0, s, a, x);
  const dim3 grid(L.evap_blocks), block(L.block);
  const size_t lds = lds_bytes(0, L.block, kXsNone, 0);
  switch (ext_of(L)) {
    case 0: hipLaunchKernelGGL((k_evap_persistent<0, false>), grid, block, lds, s, a); break;
    case kExtPhoton: hipLaunchKernelGGL((k_evap_persistent<kExtPhoton, false>), grid, block, lds, s, a); break;
    case kExtHeavy: hipLaunchKernelGGL((k_evap_persistent<kExtHeavy, false>), grid, block, lds, s, a); break;
    default: hipLaunchKernelGGL((k_evap_persistent<kExtPhoton | kExtHeavy, false>), grid, block, lds, s, a); break;
  }
  return hipGetLastError();
}

size_t vertex_slot_bytes() { return sizeof(VSlot); }
size_t vertex_stack_bytes() { return sizeof(StackEntry) * kStackDepth; }
size_t vertex_queue_words(size_t window) { return 2 * (size_t)kVStages * window; }

template <int kExt, int kStage>
static void launch_vertex_stage(const LaunchDesc& L, const KernelArgs& a, const VertexArgs& v, unsigned grid,
                                hipStream_t s) {
  if constexpr (kStage < kVRefill) {
    const size_t lds = vstage_type(kStage) == kVEvap ? lds_bytes(0, L.block, kXsNone, 0)
                                                     : lds_bytes(L.n_targets, L.block, kXsColumns, 0);
    hipLaunchKernelGGL((k_vertex<kStage, kExt>), dim3(grid), dim3(L.block), lds, s, a, v);
    launch_vertex_stage<kExt, kStage + 1>(L, a, v, grid, s);
  } else {
    hipLaunchKernelGGL(k_vertex_refill, dim3(grid), dim3(L.block), lds_bytes(L.n_targets, L.block, kXsColumns, 0), s,
                       a, v);
    hipLaunchKernelGGL(k_vertex_swap, dim3(1), dim3(64), 0, s, v);
  }
}

static void launch_vertex_group(const LaunchDesc& L, const KernelArgs& a, const VertexArgs& v, unsigned grid,
                                int cycles, hipStream_t s) {
  for (int k = 0; k < cycles; ++k) {
    switch (ext_of(L)) {
      case 0: launch_vertex_stage<0, 0>(L, a, v, grid, s); break;
      case kExtPhoton: launch_vertex_stage<kExtPhoton, 0>(L, a, v, grid, s); break;
      case kExtHeavy: launch_vertex_stage<kExtHeavy, 0>(L, a, v, grid, s); break;
      default: launch_vertex_stage<kExtPhoton | kExtHeavy, 0>(L, a, v, grid, s); break;
    }
  }
}

hipError_t launch_vertex(const LaunchDesc& L, const VertexBuf& vb, hipStream_t s) {
  const KernelArgs a = kernel_args(L);
  const uint32_t w = (uint32_t)(L.n < vb.window ? L.n : vb.window);
  VertexArgs v;
  v.slots = (VSlot*)vb.slots;
  v.stacks = (StackEntry*)vb.stacks;
  v.queues = vb.queues;
  v.ctl = vb.ctl;
  v.window = (uint32_t)vb.window;
  hipLaunchKernelGGL(k_zero_counters, dim3((L.n_seg + 63) / 64), dim3(64), 0, s, L.segs, L.n_seg, L.queue,
                     (uint32_t*)nullptr);
  hipLaunchKernelGGL(k_vertex_init, dim3((w + 255) / 256), dim3(256), 0, s, v, w);
  // grid-stride stages on at most two resident waves' worth of blocks
  const unsigned need = (w + L.block - 1) / L.block, cap = (unsigned)(2 * L.persistent_blocks);
  const unsigned grid = need < cap ? need : cap;
  hipError_t e = hipSuccess;
  // a group of cycles as one graph (kernel nodes only), built for this call's
  // arguments, replayed group after group
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  if (vb.use_graph) {
    e = hipStreamBeginCapture(vb.capture, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      launch_vertex_group(L, a, v, grid, vb.cycles_per_group, vb.capture);
      e = hipStreamEndCapture(vb.capture, &graph);
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return e;
    }
  }
  // the host reads the done flag of a group while the next group runs (two
  // flags, two events), so it waits at most one group of (then empty) cycles
  // past the end
  for (long g = 0;; ++g) {
    if (exec) e = hipGraphLaunch(exec, s);
    else launch_vertex_group(L, a, v, grid, vb.cycles_per_group, s);
    if (e == hipSuccess) e = hipMemcpyAsync(vb.h_done + (g & 1), vb.ctl + 2, sizeof(uint32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipEventRecord(vb.ev[g & 1], s);
    if (e != hipSuccess) break;
    if (g == 0) continue;
    if ((e = hipEventSynchronize(vb.ev[(g - 1) & 1])) != hipSuccess) break;
    if (vb.h_done[(g - 1) & 1]) break;
    if (g * vb.cycles_per_group > vb.max_cycles) {
      e = hipErrorLaunchTimeOut;
      break;
    }
  }
  if (exec) {
    // the last replay may still run: the executable graph goes once it is done
    (void)hipStreamSynchronize(s);
    (void)hipGraphExecDestroy(exec);
    (void)hipGraphDestroy(graph);
  }
  return e != hipSuccess ? e : hipGetLastError();
}

}  // namespace INC_KERNEL_NS
}  // namespace incdev
