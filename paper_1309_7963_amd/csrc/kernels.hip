// kernels.hip — setup kernels (Sec. 2.2, 2.3, 2.4 tables), the plain
// cascade / evaporation kernel pair (the paper's Sec. 3 organisation: one
// cascade per thread, then one de-excitation per thread) and the fused
// persistent work-queue kernel.
#include "kernels.h"

#include "event.h"

namespace incdev {

// ---------------------------------------------------------------- setup
// Semi-empirical binding energy (Sec. 2.2) in double precision: textbook
// coefficient set, measured values for d, t, 3He, alpha, zero for other A <= 4.
__device__ double semf_binding(int A, int Z) {
  if (A <= 0 || Z < 0 || Z > A) return 0.0;
  if (A <= 4) {
    if (A == 2 && Z == 1) return 2.224566;
    if (A == 3 && Z == 1) return 8.481798;
    if (A == 3 && Z == 2) return 7.718043;
    if (A == 4 && Z == 2) return 28.29566;
    return 0.0;
  }
  const int N = A - Z;
  const double a = (double)A, a13 = cbrt(a);
  double B = 15.75 * a - 17.8 * a13 * a13 - 0.711 * (double)(Z * (Z - 1)) / a13 - 23.7 * (double)((N - Z) * (N - Z)) / a;
  const double pair = 11.18 / sqrt(a);
  if (((Z | N) & 1) == 0) B += pair;
  if ((Z & 1) && (N & 1)) B -= pair;
  return B > 0.0 ? B : 0.0;
}

// Binding energies B(A, Z) for the evaporation chain, the six fragments'
// constants (mass, A^1/3, ln(g m) with spin factors g = 2, 2, 3, 2, 2, 1) and
// the per-A table of A^1/3 and ln A.
__global__ void k_bind_table(double* B, int amax, int zmax, EvapTab* et, MassTab* mt) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int zs = zmax + 1;
  if (idx < (amax + 1) * zs) B[idx] = semf_binding(idx / zs, idx % zs);
  if (idx <= kMaxA) {
    mt->a13[idx] = (float)cbrt((double)idx);
    mt->lnA[idx] = idx > 0 ? (float)log((double)idx) : 0.0f;
  }
  if (idx == 0) {
    const int fa[6] = {1, 1, 2, 3, 3, 4}, fz[6] = {0, 1, 1, 1, 2, 2};
    const double g[6] = {2.0, 2.0, 3.0, 2.0, 2.0, 1.0};
    for (int j = 0; j < 6; ++j) {
      const double b = semf_binding(fa[j], fz[j]);
      const double m = (double)fz[j] * kMassP + (double)(fa[j] - fz[j]) * kMassN - b;
      et->B[j] = b;
      et->m[j] = (float)m;
      et->a13[j] = (float)cbrt((double)fa[j]);
      et->lngm[j] = (float)log(g[j] * m);
    }
  }
}

// Fermi density of Eq. (1), c = 1.07 A^1/3, delta = 0.545, R = c + 2.5 fm,
// 15 equal shells; each shell's density is its share of the A nucleons over
// its volume (integrals by 64-panel 5-point Gauss-Legendre, double).
// Two-component Fermi gas: p_F = hbar c (3 pi^2 rho_x)^1/3, relativistic E_F.
__global__ void k_nucleus_setup(const int* AZ, NucTab* out, int uniform_density, int zero_fermi, int zero_binding) {
  __shared__ double integ[kShells];
  const int t = blockIdx.x;
  const int A = AZ[2 * t], Z = AZ[2 * t + 1];
  const double c = 1.07 * cbrt((double)A), delta = 0.545, R = c + 2.5;
  const int i = threadIdx.x;
  if (i < kShells) {
    const double gx[5] = {-0.9061798459386640, -0.5384693101056831, 0.0, 0.5384693101056831, 0.9061798459386640};
    const double gw[5] = {0.2369268850561891, 0.4786286704993665, 0.5688888888888889, 0.4786286704993665,
                          0.2369268850561891};
    const double r0 = R * i / kShells, r1 = R * (i + 1) / kShells;
    const int panels = 64;
    const double h = (r1 - r0) / panels;
    double sum = 0.0;
    for (int p = 0; p < panels; ++p) {
      const double mid = r0 + (p + 0.5) * h;
      for (int q = 0; q < 5; ++q) {
        const double r = mid + 0.5 * h * gx[q];
        sum += gw[q] * r * r / (1.0 + exp((r - c) / delta));
      }
    }
    integ[i] = 0.5 * h * sum;
  }
  __syncthreads();
  if (i < kShells) {
    double total = 0.0;
    for (int k = 0; k < kShells; ++k) total += integ[k];
    const double r0 = R * i / kShells, r1 = R * (i + 1) / kShells;
    const double pi = 3.14159265358979323846;
    double rho = (double)A * (integ[i] / total) / (4.0 / 3.0 * pi * (r1 * r1 * r1 - r0 * r0 * r0));
    if (uniform_density) rho = (double)A / (4.0 / 3.0 * pi * R * R * R);
    const double frac[2] = {(double)(A - Z) / A, (double)Z / A};
    const double mass[2] = {(double)kMassN, (double)kMassP};
    for (int sp = 0; sp < 2; ++sp) {
      const double r = rho * frac[sp];
      double pF = 197.3269804 * cbrt(3.0 * pi * pi * r);
      if (zero_fermi) pF = 0.0;
      out[t].rho[sp][i] = (float)r;
      out[t].pF[sp][i] = (float)pF;
      out[t].EF[sp][i] = (float)(pF * pF / (sqrt(pF * pF + mass[sp] * mass[sp]) + mass[sp]));
    }
    out[t].r2[i + 1] = (float)(r1 * r1);
    if (i == 0) {
      out[t].r2[0] = 0.0f;
      out[t].R = (float)R;
      double EB = semf_binding(A, Z) / A, EC = 1.44 * Z / R;
      if (zero_binding) EB = EC = 0.0;
      out[t].EB = (float)EB;
      out[t].EC = (float)EC;
      out[t].A = A;
      out[t].Z = Z;
      for (int sp = 0; sp < 2; ++sp) {
        out[t].rho[sp][15] = 0.0f;
        out[t].pF[sp][15] = 0.0f;
        out[t].EF[sp][15] = 0.0f;
      }
      for (int k = 0; k < 7; ++k) out[t].pad[k] = 0.0f;
    }
  }
  __syncthreads();
  if (i == 0) {
    // densities fall outwards: the smallest E_F is the outermost shell's, the
    // largest p_F the innermost's; scan anyway
    for (int sp = 0; sp < 2; ++sp) {
      float efmin = out[t].EF[sp][0], pfmax = out[t].pF[sp][0];
      for (int k = 1; k < kShells; ++k) {
        efmin = fminf(efmin, out[t].EF[sp][k]);
        pfmax = fmaxf(pfmax, out[t].pF[sp][k]);
      }
      out[t].EFmin[sp] = efmin;
      out[t].pFmax[sp] = pfmax;
    }
  }
}

// Free NN elastic cross-sections (Sec. 2.3, reading of the Cugnon et al.
// parameterisation): p = p_lab in GeV/c, sigma in mb; below 0.8 GeV/c the
// larger of the first two branches.
__device__ double sigma_like(double p) {
  if (p < 0.8) return fmax(34.0 * pow(p / 0.4, -2.104), 23.5 + 1000.0 * pow(p - 0.7, 4.0));
  return 1250.0 / (p + 50.0) - 4.0 * (p - 1.3) * (p - 1.3);
}
__device__ double sigma_unlike(double p) {
  if (p < 0.8) {
    const double l = log(p);
    return fmax(6.3555 * pow(p, -3.2481) * exp(-0.377 * l * l), 33.0 + 196.0 * pow(fabs(p - 0.95), 2.5));
  }
  return 31.0 / sqrt(p);
}
__device__ double slope_like(double p) {
  const double p8 = p * p * p * p * p * p * p * p;
  return 5.5 * p8 / (7.7 + p8);
}
__device__ double slope_unlike(double p) {
  if (p < 0.225) return 0.0;
  if (p < 0.6) return 16.53 * (p - 0.225);
  return -1.63 * p + 7.16;
}

__global__ void k_xs_table(XsTab* xs, float const_sigma) {
  __shared__ float sig[2][kXsNodes];
  const int k = threadIdx.x;
  const double lo = kPlo, hi = kPhi;
  if (k < kXsNodes) {
    const double p = lo * exp(log(hi / lo) * (double)k / (double)(kXsNodes - 1));
    sig[0][k] = (float)sigma_unlike(p);
    sig[1][k] = (float)sigma_like(p);
    if (const_sigma > 0.0f) sig[0][k] = sig[1][k] = const_sigma;
    xs->sig[0][k] = sig[0][k];
    xs->sig[1][k] = sig[1][k];
    xs->slope[0][k] = (float)slope_unlike(p);
    xs->slope[1][k] = (float)slope_like(p);
  }
  __syncthreads();
  if (k < 2) {
    // suffix maximum: a majorant of the interpolated sigma above each node
    float m = sig[k][kXsNodes - 1];
    for (int j = kXsNodes - 1; j >= 0; --j) {
      m = fmaxf(m, sig[k][j]);
      xs->hat[k][j] = m;
    }
  }
}

__global__ void k_fill_u64(unsigned long long* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

// ----------------------------------------------------------- event kernels
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
  unsigned long long* queue; // work-queue head (persistent kernel)
  MidState* mid;             // plain kernels: cascade -> evaporation hand-over
  RingDev ring;              // streaming output (rec == NULL: segment arrays)
  int stack_lds;             // stack entries per lane held in LDS
};

__device__ __forceinline__ bool energy_ok(float T0) { return T0 >= 20.0f && T0 <= 250.0f; }

// LDS layout of the event kernels: [n_targets NucTab][XsTab][MassTab][writer
// buffers of the block's waves][LIFO levels: per wave stack_lds x 2 x 64
// float4].  The plain evaporation kernel stages only the MassTab (n_targets =
// 0, no XsTab) and has no stack.
__device__ __forceinline__ size_t lds_mass_offset(int n_targets, bool with_xs) {
  return (size_t)n_targets * sizeof(NucTab) + (with_xs ? sizeof(XsTab) : 0);
}
// First float4 of this lane's column in the LDS stack area (each wave owns
// levels x 2 x 64 consecutive float4).
__device__ __forceinline__ int lds_stack_base(int n_targets, int levels) {
  return (int)((lds_mass_offset(n_targets, true) + sizeof(MassTab) +
                (blockDim.x / 64) * (kWriterCap * kRecWords * sizeof(uint32_t))) /
               sizeof(float4)) +
         (int)(threadIdx.x / 64) * levels * 128 + (int)(threadIdx.x % 64);
}
__device__ __forceinline__ void stage_tables(char* lds, const KernelArgs& a, int n_targets, bool with_xs) {
  uint32_t* dst = (uint32_t*)lds;
  const uint32_t* src = (const uint32_t*)a.nuc;
  for (int i = threadIdx.x; i < n_targets * (int)(sizeof(NucTab) / 4); i += blockDim.x) dst[i] = src[i];
  if (with_xs) {
    uint32_t* dx = (uint32_t*)(lds + n_targets * sizeof(NucTab));
    const uint32_t* sx = (const uint32_t*)a.xs;
    for (int i = threadIdx.x; i < (int)(sizeof(XsTab) / 4); i += blockDim.x) dx[i] = sx[i];
  }
  uint32_t* dm = (uint32_t*)(lds + lds_mass_offset(n_targets, with_xs));
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
  rng.init(a.segs[e.seg].seed, a.segs[e.seg].first_id + (a.opt.same_stream ? 0 : e.local));
}
__device__ __forceinline__ uint32_t kind_of(uint32_t k, EventRef e) { return k | ((uint32_t)e.seg << 16); }

// Plain cascade kernel: one event per thread (Sec. 3.2).  Each iteration of
// the wave loop advances every live lane by one flight segment together with
// the tentative collision and kinematics it may end in, then the wave writes
// the escaping particles through the compacted writer.
__global__ void __launch_bounds__(256) k_cascade_plain(KernelArgs a) {
  extern __shared__ __align__(16) char lds[];
  stage_tables(lds, a, a.n_targets, true);
  const NucTab* snt = (const NucTab*)lds;
  const XsTab& sxs = *(const XsTab*)(lds + a.n_targets * sizeof(NucTab));
  uint32_t* wbuf = (uint32_t*)(lds + lds_mass_offset(a.n_targets, true) + sizeof(MassTab)) +
                   (threadIdx.x / 64) * (kWriterCap * kRecWords);
  int fill = 0;

  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool live = i < a.n;
  float T0 = 0.0f;
  int tgt = 0;
  EventRef er = {0, 0};
  Rng rng;
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
  c.stk_base = lds_stack_base(a.n_targets, a.stack_lds);
  c.stk_levels = a.stack_lds;

  while (__any(live)) {
    Emit em;
    em.on = false;
    if (live) {
      int st = flight_step(c, stk, rng, nt, sxs, a.opt, T0, em);
      if (st == kStTent) st = tent_step(c, rng, nt, sxs, a.opt);
      if (st == kStKin) st = kin_step(c, stk, rng, nt, sxs, a.opt);
      if (st == kStDone) {
        const Nucleus r = cascade_residual(c, nt, T0);
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
    writer_append(wbuf, fill, a.segs, a.ring, em.on, er.local, kind_of(em.kind, er), em.T, em.u);
  }
  writer_flush(wbuf, fill, a.segs, a.ring);
}

// Plain evaporation kernel: one de-excitation per thread (Sec. 3.3), same
// random stream continued after the cascade's draws.
__global__ void __launch_bounds__(256) k_evap_plain(KernelArgs a) {
  extern __shared__ __align__(16) char lds[];
  stage_tables(lds, a, 0, false);
  const MassTab& smt = *(const MassTab*)lds;
  uint32_t* wbuf = (uint32_t*)(lds + sizeof(MassTab)) + (threadIdx.x / 64) * (kWriterCap * kRecWords);
  int fill = 0;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool live = i < a.n;
  MidState m = {};
  Nucleus nu = {0, 0, 0.0f, {0.0f, 0.0f, 0.0f}};
  Rng rng;
  EventRef er = {0, 0};
  int nsec = 0, flags = 0;
  if (live) {
    er = event_ref(a, i);
    inc_residual* res = a.segs[er.seg].res + er.local;
    m = a.mid[i];
    flags = m.flags;
    if (flags & kFlagRange) {
      write_residual(res, nu, 0.0f, 0, flags, 0, 0);
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
        live = false;
      }
    }
  }
  while (__any(live)) {
    Emit em;
    em.on = false;
    if (live) {
      if (evap_step(nu, rng, a.bind, a.evap, smt, em)) {
        write_residual(a.segs[er.seg].res + er.local, nu, m.E, nsec, flags, m.ncoll, m.nretry);
        live = false;
      } else {
        ++nsec;
      }
    }
    writer_append(wbuf, fill, a.segs, a.ring, em.on, er.local, kind_of(em.kind, er), em.T, em.u);
  }
  writer_flush(wbuf, fill, a.segs, a.ring);
}

// Persistent fused kernel.  Every wave keeps 64 events in flight; finished
// lanes refill from a global work queue (one atomic per 64 events per wave).
// Each iteration the wave advances the lanes of ONE state (FLIGHT, TENT, KIN
// or EVAP), chosen by ballot: a deeper state runs once enough lanes wait in it
// (kin / tent / evap thresholds), else FLIGHT, else whatever state has lanes.
// Lanes in other states wait, so every step runs with many lanes together;
// each lane still consumes its own random stream in order, so results do not
// depend on the schedule.
constexpr int kChunk = 64;

// 3 waves per SIMD (<= 168 VGPRs): the lane scheduler needs many events in
// flight per CU more than it needs extra registers.
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) k_persistent(KernelArgs a) {
  extern __shared__ __align__(16) char lds[];
  stage_tables(lds, a, a.n_targets, true);
  const NucTab* snt = (const NucTab*)lds;
  const XsTab& sxs = *(const XsTab*)(lds + a.n_targets * sizeof(NucTab));
  const MassTab& smt = *(const MassTab*)(lds + lds_mass_offset(a.n_targets, true));
  uint32_t* wbuf = (uint32_t*)(lds + lds_mass_offset(a.n_targets, true) + sizeof(MassTab)) +
                   (threadIdx.x / 64) * (kWriterCap * kRecWords);
  int fill = 0;

  unsigned long long chunk_next = 0, chunk_end = 0;
  bool exhausted = false;
  int st = kStDone;
  EventRef er = {0, 0};
  float T0 = 0.0f;
  int tgt = 0, nsec = 0;
  float Ex_casc = 0.0f;
  Rng rng;
  Cascade c;
  Nucleus nu = {0, 0, 0.0f, {0.0f, 0.0f, 0.0f}};
  StackEntry stk[kStackDepth];
  c.stk_base = lds_stack_base(a.n_targets, a.stack_lds);
  c.stk_levels = a.stack_lds;

  for (;;) {
    // ---- refill finished lanes from the work queue
    const uint64_t need = __ballot(st == kStDone);
    if (need && !exhausted) {
      if (chunk_next == chunk_end) {
        unsigned long long base = 0;
        if (lane_id() == 0) base = atomicAdd(a.queue, (unsigned long long)kChunk);
        base = __shfl(base, 0);
        chunk_next = base;
        chunk_end = base + kChunk < a.n ? base + kChunk : a.n;
        if (base >= a.n) {
          exhausted = true;
          chunk_next = chunk_end = a.n;
        }
      }
      const unsigned long long avail = chunk_end - chunk_next;
      const uint32_t r = rank_in(need);
      if (st == kStDone && r < avail) {
        const size_t ev = (size_t)(chunk_next + r);
        er = event_ref(a, ev);
        T0 = a.T0[ev];
        tgt = a.tidx ? (int)a.tidx[ev] : 0;
        if (!energy_ok(T0) || tgt >= a.n_targets) {
          tgt = 0;
          const Nucleus z = {0, 0, 0.0f, {0.0f, 0.0f, 0.0f}};
          write_residual(a.segs[er.seg].res + er.local, z, 0.0f, 0, kFlagRange, 0, 0);
          atomicAdd(&a.segs[er.seg].counters[1], 1ull);
        } else {
          init_stream(rng, a, er);
          cascade_init(c, snt[tgt]);
          nsec = 0;
          st = kStFlight;
        }
      }
      const unsigned long long cnt = (unsigned long long)__popcll(need);
      chunk_next += cnt < avail ? cnt : avail;
    }
    if (exhausted && st == kStDone) st = kStIdle;
    const int nF = __popcll(__ballot(st == kStFlight));
    const int nT = __popcll(__ballot(st == kStTent));
    const int nK = __popcll(__ballot(st == kStKin));
    const int nE = __popcll(__ballot(st == kStEvap));
    if (nF + nT + nK + nE == 0) {
      if (exhausted) break;
      continue;
    }
    // ---- state selection (wave-uniform)
    int run;
    if (nK >= a.opt.kin_threshold) run = kStKin;
    else if (nT >= a.opt.tent_threshold) run = kStTent;
    else if (nE >= a.opt.evap_threshold) run = kStEvap;
    else if (nF) run = kStFlight;
    else if (nK) run = kStKin;
    else if (nT) run = kStTent;
    else run = kStEvap;

    Emit em;
    em.on = false;
    if (run == kStEvap) {
      if (st == kStEvap) {
        if (evap_step(nu, rng, a.bind, a.evap, smt, em)) {
          write_residual(a.segs[er.seg].res + er.local, nu, Ex_casc, nsec, c.flags, c.ncoll, c.nretry);
          if (c.flags) atomicAdd(&a.segs[er.seg].counters[1], 1ull);
          st = kStDone;
        } else {
          ++nsec;
        }
      }
    } else if (st == run) {
      const NucTab& nt = snt[tgt];
      int ns;
      if (run == kStFlight) ns = flight_step(c, stk, rng, nt, sxs, a.opt, T0, em);
      else if (run == kStTent) ns = tent_step(c, rng, nt, sxs, a.opt);
      else ns = kin_step(c, stk, rng, nt, sxs, a.opt);
      if (em.on) ++nsec;
      if (ns == kStDone) {
        nu = cascade_residual(c, nt, T0);
        Ex_casc = nu.E;
        if (nu.A <= 0) c.flags |= kFlagEmpty;
        if (nu.A <= 0 || a.opt.no_evaporation) {
          write_residual(a.segs[er.seg].res + er.local, nu, Ex_casc, nsec, c.flags, c.ncoll, c.nretry);
          if (c.flags) atomicAdd(&a.segs[er.seg].counters[1], 1ull);
          st = kStDone;
        } else {
          st = kStEvap;
        }
      } else {
        st = ns;
      }
    }
    writer_append(wbuf, fill, a.segs, a.ring, em.on, er.local, kind_of(em.kind, er), em.T, em.u);
  }
  writer_flush(wbuf, fill, a.segs, a.ring);
}

// Zero the segments' counters and the work-queue head (a fill kernel rather
// than a memset, so the launch sequence stays capturable in a graph).
__global__ void k_zero_counters(const Segment* segs, int n_seg, unsigned long long* queue) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_seg) {
    segs[i].counters[0] = 0ull;
    segs[i].counters[1] = 0ull;
  }
  if (i == 0) *queue = 0ull;
}

// Copy one segment description (a kernel argument) into device memory.
__global__ void k_set_segment(Segment s, Segment* dst) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *dst = s;
}

}  // namespace incdev

// ================================================================ launchers
using namespace incdev;

size_t inc_lds_bytes(int n_targets, int block, bool with_xs, int stack_levels) {
  return (size_t)n_targets * sizeof(NucTab) + (with_xs ? sizeof(XsTab) : 0) + sizeof(MassTab) +
         (size_t)(block / 64) * kWriterCap * kRecWords * sizeof(uint32_t) +
         (size_t)stack_levels * 2 * block * sizeof(float4);
}

int inc_stack_levels(int mode, int n_targets, int block, int waves_per_cu) {
  int dev = 0, lds_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) != hipSuccess ||
      lds_cu <= 0)
    return 0;
  const size_t base = inc_lds_bytes(n_targets, block, true, 0);
  int occ = 0;
  const void* fn = mode == INC_MODE_PLAIN ? (const void*)k_cascade_plain : (const void*)k_persistent;
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

hipError_t inc_launch_setup(const int* d_AZ, int n_targets, NucTab* d_nuc, XsTab* d_xs, double* d_B, int amax,
                            int zmax, EvapTab* d_evap, MassTab* d_mass, const inc_options& o, hipStream_t s) {
  hipLaunchKernelGGL(k_nucleus_setup, dim3(n_targets), dim3(64), 0, s, d_AZ, d_nuc, o.uniform_density, o.zero_fermi,
                     o.zero_binding);
  hipLaunchKernelGGL(k_xs_table, dim3(1), dim3(kXsNodes), 0, s, d_xs, o.const_sigma_mb);
  const int cells = (amax + 1) * (zmax + 1) > kMaxA + 1 ? (amax + 1) * (zmax + 1) : kMaxA + 1;
  hipLaunchKernelGGL(k_bind_table, dim3((cells + 255) / 256), dim3(256), 0, s, d_B, amax, zmax, d_evap, d_mass);
  return hipGetLastError();
}

hipError_t inc_upload_segment(const Segment& seg, Segment* d_slot, hipStream_t s) {
  hipLaunchKernelGGL(k_set_segment, dim3(1), dim3(64), 0, s, seg, d_slot);
  return hipGetLastError();
}

hipError_t inc_launch_events(const LaunchDesc& L, hipStream_t s) {
  KernelArgs a;
  a.nuc = L.nuc;
  a.n_targets = L.n_targets;
  a.xs = L.xs;
  a.mass = L.mass;
  a.bind = {L.bind, L.zmax + 1, L.amax, L.zmax};
  a.evap = L.evap;
  a.opt.no_pauli = L.opt.no_pauli;
  a.opt.no_evaporation = L.opt.no_evaporation;
  a.opt.stop_after_first = L.opt.stop_after_first;
  a.opt.const_sigma_mb = L.opt.const_sigma_mb;
  a.opt.fixed_b = L.fixed_b_set ? L.opt.fixed_b : -1.0f;
  a.opt.evap_threshold = L.evap_threshold;
  a.opt.tent_threshold = L.tent_threshold;
  a.opt.kin_threshold = L.kin_threshold;
  a.opt.same_stream = L.opt.same_stream;
  a.n = L.n;
  a.tidx = L.tidx;
  a.T0 = L.T0;
  a.segs = L.segs;
  a.n_seg = L.n_seg;
  a.queue = L.queue;
  a.mid = L.mid;
  a.ring = L.ring;
  a.stack_lds = L.stack_lds;
  hipLaunchKernelGGL(k_zero_counters, dim3((L.n_seg + 63) / 64), dim3(64), 0, s, L.segs, L.n_seg, L.queue);
  const int block = L.block;
  if (L.mode == INC_MODE_PLAIN) {
    const unsigned grid = (unsigned)((L.n + block - 1) / block);
    hipLaunchKernelGGL(k_cascade_plain, dim3(grid), dim3(block), inc_lds_bytes(L.n_targets, block, true, L.stack_lds),
                       s, a);
    hipLaunchKernelGGL(k_evap_plain, dim3(grid), dim3(block), inc_lds_bytes(0, block, false, 0), s, a);
  } else {
    hipLaunchKernelGGL(k_persistent, dim3(L.persistent_blocks), dim3(block),
                       inc_lds_bytes(L.n_targets, block, true, L.stack_lds), s, a);
  }
  return hipGetLastError();
}
