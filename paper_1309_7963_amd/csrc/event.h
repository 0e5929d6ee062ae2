// event.h — per-lane state machines of one non-elastic event: the
// intranuclear cascade (Sec. 2.3) and the evaporation (Sec. 2.4).
//
// A lane is always in one of a few states and advances by one bounded step per
// call: START (begin a flight: the entry of a pass, or the next particle from
// the stack after an escape), FLIGHT (one flight segment, ending at a shell
// boundary, at a tentative collision point or at an escape; no random draws),
// TENT (the tentative collision: target species and momentum, p_lab, accept
// test), KIN (the accepted collision: CM angle, boosts, Pauli test, cutoff,
// stack), EVAP (one evaporation emission).  The kernels keep the whole wave
// converged at the writer after every step, and the persistent kernel picks
// per iteration which state the wave advances, so that each step runs with
// many lanes together and the rare paths (entry, stack pop) do not ride along
// with every flight segment.
#pragma once

#include "device.h"

namespace incdev {

enum : int {
  kStIdle = 0,    // no event (queue exhausted)
  kStFlight = 1,
  kStTent = 2,
  kStKin = 3,
  kStEvap = 4,
  kStDone = 5,    // event finished, lane needs a new one
  kStStart = 6,   // begin a flight (entry of a pass, or pop after an escape)
};

// Cascade state of one event (registers).  The LIFO of pending products
// is split between LDS and a private array owned by the kernel.
struct Cascade {
  V3 pos, dir;
  float eps;       // T - E_F(local): invariant under refraction
  int sp;          // 0 n, 1 p
  int shell;       // 0..14
  float tau;       // remaining optical depth
  float sh0, sh1;  // majorant cross-sections (fm^2) against n, p
  float Ex;        // accumulated excitation energy
  V3 pesc;         // sum of escaped momenta
  int nesc0, nesc1, avail0, avail1;
  int ncoll, nretry, nseg, flags, top;
  uint32_t hsh;    // h = 3 h + shell + 1 over the tentative collisions (path fingerprint)
  int started;
  V3 pt;           // target momentum of the pending collision (TENT -> KIN)
  float ptm;       // its magnitude, as sampled
  int ytgt;        // target species of the pending collision
  int stk_base, stk_levels;  // LDS part of the LIFO (set by the kernel)
};

// Residual nucleus entering / leaving the evaporation.
struct Nucleus {
  int A, Z;
  float E;   // excitation energy
  V3 P;      // momentum
};

// LIFO of pending products (depth kStackDepth).  The lowest `stk_levels`
// entries of each lane sit in LDS, interleaved over the 64 lanes of the wave
// (entry t, half h of the lane at float4 index stk_base + (2 t + h) * 64 of the
// dynamic LDS), so a wave's pushes and pops are bank-conflict-free and never
// leave the CU; deeper entries go to the kernel's private array.  An entry is
// (pos, dir.x) and (dir.y, dir.z, eps, sp | shell << 1).
extern __shared__ __align__(16) float4 lds_f4[];

struct StackEntry {
  float v[8];
};

__device__ __forceinline__ void push(StackEntry* stk, Cascade& c, V3 pos, V3 dir, float eps, int sp) {
  const int t = c.top++;
  const float4 lo = make_float4(pos.x, pos.y, pos.z, dir.x);
  const float4 hi = make_float4(dir.y, dir.z, eps, __int_as_float(sp | (c.shell << 1)));
  if (t < c.stk_levels) {
    lds_f4[c.stk_base + 2 * t * 64] = lo;
    lds_f4[c.stk_base + (2 * t + 1) * 64] = hi;
  } else {
    float* v = stk[t].v;
    v[0] = lo.x; v[1] = lo.y; v[2] = lo.z; v[3] = lo.w;
    v[4] = hi.x; v[5] = hi.y; v[6] = hi.z; v[7] = hi.w;
  }
}
__device__ __forceinline__ void pop(StackEntry* stk, Cascade& c) {
  const int t = --c.top;
  float4 lo, hi;
  if (t < c.stk_levels) {
    lo = lds_f4[c.stk_base + 2 * t * 64];
    hi = lds_f4[c.stk_base + (2 * t + 1) * 64];
  } else {
    const float* v = stk[t].v;
    lo = make_float4(v[0], v[1], v[2], v[3]);
    hi = make_float4(v[4], v[5], v[6], v[7]);
  }
  c.pos = {lo.x, lo.y, lo.z};
  c.dir = {lo.w, hi.x, hi.y};
  c.eps = hi.z;
  const int k = __float_as_int(hi.w);
  c.sp = k & 1;
  c.shell = k >> 1;
}

__device__ __forceinline__ void cascade_init(Cascade& c, const NucTab& nt) {
  c.Ex = 0.0f;
  c.pesc = {0.0f, 0.0f, 0.0f};
  c.nesc0 = c.nesc1 = 0;
  c.avail0 = nt.A - nt.Z;  // the projectile proton is out of the sea
  c.avail1 = nt.Z;
  c.ncoll = c.nretry = c.nseg = c.flags = c.top = 0;
  c.hsh = 0u;
  c.started = 0;
}

// Entry (reading): impact parameter uniform over the disc of radius R,
// incidence along +z, inward refraction at R; then the first optical depth.
template <class XS, class O>
__device__ __forceinline__ void cascade_entry(Cascade& c, Rng& rng, const NucTab& nt, const XS& xs,
                                              const O& o, float T0) {
  const float ub = rng.next();
  const float uphi = rng.next();
  float b, z;
  if (o.fixed_b >= 0.0f) {
    b = o.fixed_b;
    z = -sqrtf(fmaxf(0.0f, nt.R * nt.R - b * b));
  } else {
    b = nt.R * sqrtf(ub);
    z = -nt.R * sqrtf(1.0f - ub);
  }
  float sp, cp;
  sincospif(2.0f * uphi, &sp, &cp);
  c.pos = {b * cp, b * sp, z};
  c.dir = {0.0f, 0.0f, 1.0f};
  c.eps = T0 + nt.EB;
  c.sp = 1;
  c.shell = kShells - 1;
  const float r = sqrtf(dot3(c.pos, c.pos));
  const V3 n = r > 0.0f ? scale(1.0f / r, c.pos) : V3{0.0f, 0.0f, -1.0f};
  refract(c.dir, n, T0, c.eps + nt.EF[1][kShells - 1], kMassP);
  majorant(nt, xs, o, c.sp, c.eps, c.sh0, c.sh1);
  c.tau = -logf(rng.next());
  c.started = 1;
}

// Capture (cutoff, Sec. 2.3): the particle stays, its excess energy heats the
// nucleus and it rejoins the Fermi sea.
__device__ __forceinline__ void capture(Cascade& c, float eps, int sp) {
  c.Ex += eps;
  if (sp) ++c.avail1; else ++c.avail0;
}

// Take the next particle from the stack or end the cascade.  Returns false
// when the cascade is over.
template <class XS, class O>
__device__ __forceinline__ bool next_particle(Cascade& c, StackEntry* stk, Rng& rng, const NucTab& nt,
                                              const XS& xs, const O& o) {
  if (c.top == 0) return false;
  pop(stk, c);
  majorant(nt, xs, o, c.sp, c.eps, c.sh0, c.sh1);
  c.tau = -logf(rng.next());
  return true;
}

struct Emit {
  bool on;
  uint32_t kind;
  float T;
  V3 u;
};

__device__ __forceinline__ float flight_weight(const Cascade& c, const NucTab& nt, int y, int s) {
  return y ? (c.avail1 > 0 ? nt.rho[1][s] * c.sh1 : 0.0f) : (c.avail0 > 0 ? nt.rho[0][s] * c.sh0 : 0.0f);
}

// START: begin the next flight.  A pass that has not started enters the
// nucleus (impact parameter, refraction, majorant, first optical depth);
// otherwise the particle in hand has escaped and the next one comes from the
// stack (kStDone when it is empty).  Draws at most 3 uniforms.
template <class XS, class O>
__device__ __forceinline__ int start_step(Cascade& c, StackEntry* stk, Rng& rng, const NucTab& nt, const XS& xs,
                                          const O& o, float T0) {
  rng.ensure(3);
  if (!c.started) {
    cascade_entry(c, rng, nt, xs, o, T0);
    return kStFlight;
  }
  return next_particle(c, stk, rng, nt, xs, o) ? kStFlight : kStDone;
}

// FLIGHT: one flight segment (null-collision flight, reading of the mean free
// path): the segment ends at a tentative collision point (-> TENT) or at a
// shell boundary, where the particle is refracted, reflected or escapes (Sec.
// 2.3).  An escape emits the particle and returns kStStart (next particle); an
// escape before any collision is a transparent pass, retried from the entry
// (Sec. 2.1), also through kStStart.  kStDone: the segment guard ended the
// cascade.  No random draws.
__device__ __forceinline__ int flight_core(Cascade& c, StackEntry* stk, const NucTab& nt, Emit& em) {
  em.on = false;
  if (c.nseg >= kMaxSegments) {
    // segment guard: capture everything still moving
    c.flags |= kFlagSegments;
    capture(c, c.eps, c.sp);
    while (c.top > 0) {
      pop(stk, c);
      capture(c, c.eps, c.sp);
    }
    return kStDone;
  }
  ++c.nseg;
  const int s = c.shell;
  const float lam = flight_weight(c, nt, 0, s) + flight_weight(c, nt, 1, s);
  const float xd = dot3(c.pos, c.dir);
  const V3 cx = {c.pos.y * c.dir.z - c.pos.z * c.dir.y, c.pos.z * c.dir.x - c.pos.x * c.dir.z,
                 c.pos.x * c.dir.y - c.pos.y * c.dir.x};
  const float b2 = dot3(cx, cx);
  const float rin2 = nt.r2[s], rout2 = nt.r2[s + 1];
  // next crossing: the inner sphere when the ray meets it, else the outer one
  // (one square root whichever way the lanes of the wave go)
  const bool inward = s > 0 && xd < 0.0f && b2 < rin2;
  const float root = sqrtf(fmaxf(0.0f, (inward ? rin2 : rout2) - b2));
  const float t = fmaxf(0.0f, -xd + (inward ? -root : root));
  const int dest = inward ? s - 1 : s + 1;
  if (c.tau < lam * t) {
    c.pos = axpy(c.tau / lam, c.dir, c.pos);
    return kStTent;
  }
  // ---- boundary crossing (Sec. 2.3 refraction / reflection)
  c.tau -= lam * t;
  c.pos = axpy(t, c.dir, c.pos);
  const V3 n = unit(c.pos);
  const float m = nucleon_mass(c.sp);
  const float T_from = c.eps + nt.EF[c.sp][s];
  if (dest == kShells) {
    const float T_out = c.eps - nt.EB;
    if (refract(c.dir, n, T_from, T_out, m)) {
      if (c.ncoll == 0) {
        // transparent pass: not a non-elastic event, try again (Sec. 2.1)
        ++c.nretry;
        c.started = 0;
        return kStStart;
      }
      const float p = sqrtf(T_out * T_out + 2.0f * T_out * m);
      c.pesc = axpy(p, c.dir, c.pesc);
      if (c.sp) ++c.nesc1; else ++c.nesc0;
      em.on = true;
      em.kind = (uint32_t)c.sp;  // stage 0
      em.T = T_out;
      em.u = c.dir;
      return kStStart;
    }
  } else if (refract(c.dir, n, T_from, c.eps + nt.EF[c.sp][dest], m)) {
    c.shell = dest;
  }
  return kStFlight;
}

// START and FLIGHT as one call (the plain kernel): the entry when the pass has
// not started, one segment, and after an escape the next particle.  Returns
// kStFlight, kStTent or kStDone; a transparent pass returns kStFlight with the
// entry left for the next call.
template <class XS, class O>
__device__ __forceinline__ int flight_step(Cascade& c, StackEntry* stk, Rng& rng, const NucTab& nt, const XS& xs,
                                           const O& o, float T0, Emit& em) {
  if (!c.started) start_step(c, stk, rng, nt, xs, o, T0);
  int st = flight_core(c, stk, nt, em);
  if (st == kStStart) st = c.started ? start_step(c, stk, rng, nt, xs, o, T0) : kStFlight;
  return st;
}

// Invariants of the pair (x, y) used by TENT and KIN.
struct Pair {
  float mx, my, Tx, Tt, rs, irs, pstar, plab;
  V3 px;
};
__device__ __forceinline__ Pair pair_of(const Cascade& c, const NucTab& nt, int y) {
  Pair q;
  const int s = c.shell;
  q.mx = nucleon_mass(c.sp);
  q.my = nucleon_mass(y);
  q.Tx = c.eps + nt.EF[c.sp][s];
  q.px = scale(sqrtf(q.Tx * q.Tx + 2.0f * q.Tx * q.mx), c.dir);
  q.Tt = kinetic_of(c.ptm, q.my);
  const float Q = 2.0f * (q.Tx * q.Tt + q.Tx * q.my + q.Tt * q.mx - dot3(q.px, c.pt));
  const float ss = (q.mx + q.my) * (q.mx + q.my) + Q;
  q.rs = sqrtf(ss);
  q.irs = 1.0f / q.rs;
  q.pstar = 0.5f * sqrtf(Q * (Q + 4.0f * q.mx * q.my)) * q.irs;
  q.plab = q.pstar * q.rs * inv_nucleon_mass(y);
  return q;
}

// TENT: the tentative collision.  Target species in proportion to
// rho_y sigma_hat_xy, target momentum uniform in the local Fermi sphere
// (Sec. 2.2), accept with sigma(p_lab) / sigma_hat.  A rejected (null)
// collision draws a fresh optical depth and the flight goes on (-> FLIGHT);
// an accepted one goes to KIN.  Draws at most 6 uniforms.
template <class XS, class O>
__device__ __forceinline__ int tent_step(Cascade& c, Rng& rng, const NucTab& nt, const XS& xs, const O& o) {
  rng.ensure(6);
  const int s = c.shell;
  c.hsh = c.hsh * 3u + (uint32_t)(s + 1);
  const float w0 = flight_weight(c, nt, 0, s), w1 = flight_weight(c, nt, 1, s);
  const int y = (w0 > rng.next() * (w0 + w1)) ? 0 : 1;
  const float ptm = nt.pF[y][s] * cbrtf(rng.next());
  const float ct = 2.0f * rng.next() - 1.0f;
  const float st = sqrtf(fmaxf(0.0f, 1.0f - ct * ct));
  float sph, cph;
  sincospif(2.0f * rng.next(), &sph, &cph);
  c.pt = {ptm * st * cph, ptm * st * sph, ptm * ct};
  c.ptm = ptm;
  c.ytgt = y;
  const Pair q = pair_of(c, nt, y);
  int k;
  float f;
  xs_coord(q.plab * 1e-3f, k, f);
  const int like = (c.sp == y);
  const float sig = (o.const_sigma_mb > 0.0f ? o.const_sigma_mb : xs_sig(xs, like, k, f)) * kMbToFm2;
  const float shy = y ? c.sh1 : c.sh0;
  if (!(rng.next() * shy < sig)) {  // u < sigma / sigma_hat
    c.tau = -logf(rng.next());
    return kStFlight;
  }
  return kStKin;
}

// KIN: elastic scattering in the CM frame (Sec. 2.3), dsigma/dt ~ exp(b t),
// boosts to the lab, Pauli test on both products, hole energy, cutoff
// capture, LIFO push of the struck nucleon.  Returns the next state (kStDone
// when the cascade is over).  Draws at most 4 uniforms.
template <class XS, class O>
__device__ __forceinline__ int kin_step(Cascade& c, StackEntry* stk, Rng& rng, const NucTab& nt, const XS& xs,
                                        const O& o) {
  rng.ensure(4);
  const int s = c.shell;
  const int y = c.ytgt;
  const Pair q = pair_of(c, nt, y);
  const int like = (c.sp == y);
  const float u_th = rng.next();
  const float u_ph = rng.next();
  const float b = slope_b(like, q.plab * 1e-3f);
  const V3 P = {q.px.x + c.pt.x, q.px.y + c.pt.y, q.px.z + c.pt.z};
  const V3 u = scale(q.irs, P);
  const float g = (q.Tx + q.Tt + q.mx + q.my) * q.irs;
  const float ig1 = 1.0f / (g + 1.0f);
  const V3 qcm = axpy(dot3(u, q.px) * ig1 - (q.Tx + q.mx), u, q.px);
  const V3 a = unit(qcm);
  const float kk = 2.0f * b * (q.pstar * 1e-3f) * (q.pstar * 1e-3f);
  float yy = (kk < 1e-6f) ? 2.0f * u_th : -log1p_acc(u_th * expm1f(-2.0f * kk)) / kk;
  yy = fminf(fmaxf(yy, 0.0f), 2.0f);
  const float cth = 1.0f - yy;
  const float sth = sqrtf(fmaxf(0.0f, yy * (2.0f - yy)));
  const V3 nn = rotate(a, cth, sth, u_ph);
  V3 qx, qt;
  float Txn, Ttn;
  const float uu1 = dot3(u, u) * ig1;
  boost_out(scale(q.pstar, nn), q.mx, u, g, ig1, uu1, qx, Txn);
  boost_out(scale(-q.pstar, nn), q.my, u, g, ig1, uu1, qt, Ttn);
  if (like && rng.next() < 0.5f) {
    const V3 tq = qx;
    qx = qt;
    qt = tq;
    Txn = Ttn;
  }
  // Pauli (Sec. 2.3): both products above their local Fermi energy.  The
  // struck product's excess energy follows from energy conservation.
  const float EFx = nt.EF[c.sp][s], EFy = nt.EF[y][s];
  const float h = fmaxf(0.0f, EFy - q.Tt);
  const float ex = Txn - EFx;
  const float ey = c.eps - ex - h;
  if (!o.no_pauli && !(ex > 0.0f && ey > 0.0f)) {
    c.tau = -logf(rng.next());
    return kStFlight;
  }
  ++c.ncoll;
  if (y) --c.avail1; else --c.avail0;
  c.Ex += h;
  const V3 dx = unit(qx), dy = unit(qt);
  const int spx = c.sp;
  if (o.stop_after_first) {
    capture(c, ex, spx);
    capture(c, ey, y);
    while (c.top > 0) {
      pop(stk, c);
      capture(c, c.eps, c.sp);
    }
    return kStDone;
  }
  const bool tx = ex >= nt.EB + (spx ? nt.EC : 0.0f);
  const bool ty = ey >= nt.EB + (y ? nt.EC : 0.0f);
  if (!tx) capture(c, ex, spx);
  if (!ty) capture(c, ey, y);
  if (tx && ty) {
    if (c.top >= kStackDepth) {
      c.flags |= kFlagStack;
      capture(c, ey, y);
    } else {
      push(stk, c, c.pos, dy, ey, y);
    }
    c.dir = dx;
    c.eps = ex;
  } else if (tx) {
    c.dir = dx;
    c.eps = ex;
  } else if (ty) {
    c.dir = dy;
    c.eps = ey;
    c.sp = y;
  } else {
    return next_particle(c, stk, rng, nt, xs, o) ? kStFlight : kStDone;
  }
  majorant(nt, xs, o, c.sp, c.eps, c.sh0, c.sh1);
  c.tau = -logf(rng.next());
  return kStFlight;
}

// Residual after the cascade (Sec. 2.3, excitation by energy conservation).
__device__ __forceinline__ Nucleus cascade_residual(const Cascade& c, const NucTab& nt, float T0) {
  Nucleus r;
  r.A = nt.A + 1 - c.nesc0 - c.nesc1;
  r.Z = nt.Z + 1 - c.nesc1;
  r.E = c.Ex;
  const float p0 = sqrtf(T0 * T0 + 2.0f * T0 * kMassP);
  r.P = {-c.pesc.x, -c.pesc.y, p0 - c.pesc.z};
  return r;
}


// Evaporation options compiled into a kernel instantiation (bits).
constexpr int kExtPhoton = 1;  // the photon channel (R19)
constexpr int kExtHeavy = 2;   // the heavier fragments (R20)

// EVAP: one evaporation step (Sec. 2.4, Weisskopf-Ewing reading).  Returns true
// when no channel is open (the nucleus is final).  Draws at most 4 uniforms.
// kExt: the optional channels that compete (the photon, channel 6; the
// heavier fragments, channels 7-26), each a separate instantiation, so that
// the paper's model compiles without any of their code.
template <int kExt>
__device__ __forceinline__ bool evap_step(Nucleus& nu, Rng& rng, const BindTab& bt, const EvapTab& et,
                                          const MassTab& mt, Emit& em) {
  constexpr bool kPhoton = (kExt & kExtPhoton) != 0;
  constexpr bool kHvy = (kExt & kExtHeavy) != 0;
  em.on = false;
  rng.ensure(4);
  constexpr int fa[6] = {1, 1, 2, 3, 3, 4};
  constexpr int fz[6] = {0, 1, 1, 1, 2, 2};
  // this nucleus's channel constants (S_j = +inf for a missing daughter)
  const ChanRow& row = bt.chan[nu.A * bt.zstride + nu.Z];
  float lw[6], U[6], V[6], Y[6];
  float lmax = -INFINITY;
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    lw[j] = -INFINITY;
    Y[j] = 0.0f;
    V[j] = row.V[j];
    U[j] = nu.E - row.S[j] - V[j];
    if (U[j] > 0.0f) {
      const int Ad = nu.A - fa[j];
      const float a = (float)Ad * 0.125f;
      Y[j] = 2.0f * sqrtf(a * U[j]);
      lw[j] = row.P[j] + log_width_integral(Y[j], mt.lnA[Ad]);
      lmax = fmaxf(lmax, lw[j]);
    }
  }
  // the optional photon channel (channel 6, after the particles): A and Z
  // stay, the level density is the nucleus's own (a = A/8)
  float lwg = -INFINITY, Yg = 0.0f;
  if constexpr (kPhoton) {
    if (nu.E > kPhotonMin && row.lg > -INFINITY) {
      Yg = 2.0f * sqrtf((float)nu.A * 0.125f * nu.E);
      lwg = row.lg + log_photon_integral(Yg, nu.E);
      lmax = fmaxf(lmax, lwg);
    }
  }
  // the optional heavier fragments (channels 7-26), the particles' width form
  constexpr int ha[kHeavy] = INC_HEAVY_A;
  constexpr int hz[kHeavy] = INC_HEAVY_Z;
  float wh[kHvy ? kHeavy : 1];
  if constexpr (kHvy) {
    const HeavyRow& hrow = bt.heavy[nu.A * bt.zstride + nu.Z];
#pragma unroll
    for (int i = 0; i < kHeavy; ++i) {
      wh[i] = -INFINITY;
      const float Uh = nu.E - hrow.S[i] - hrow.V[i];
      if (Uh > 0.0f) {
        const int Ad = nu.A - ha[i];
        wh[i] = hrow.P[i] + log_width_integral(2.0f * sqrtf((float)Ad * 0.125f * Uh), mt.lnA[Ad]);
        lmax = fmaxf(lmax, wh[i]);
      }
    }
  }
  if (lmax == -INFINITY) return true;
  float w[6], total = 0.0f;
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    w[j] = lw[j] == -INFINITY ? 0.0f : expf(lw[j] - lmax);
    total += w[j];
  }
  float wg = 0.0f;
  if constexpr (kPhoton) {
    wg = lwg == -INFINITY ? 0.0f : expf(lwg - lmax);
    total += wg;
  }
  if constexpr (kHvy) {
#pragma unroll
    for (int i = 0; i < kHeavy; ++i) {
      wh[i] = wh[i] == -INFINITY ? 0.0f : expf(wh[i] - lmax);
      total += wh[i];
    }
  }
  const float uc = rng.next() * total;
  int j = -1;
  float cum = 0.0f;
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    cum += w[i];
    if (j < 0 && w[i] > 0.0f && cum > uc) j = i;
  }
  if constexpr (kPhoton) {
    cum += wg;
    if (j < 0 && wg > 0.0f && cum > uc) j = 6;
  }
  if constexpr (kHvy) {
#pragma unroll
    for (int i = 0; i < kHeavy; ++i) {
      cum += wh[i];
      if (j < 0 && wh[i] > 0.0f && cum > uc) j = 7 + i;
    }
  }
  if (j < 0) {
    // rounding at the top: the last open channel
#pragma unroll
    for (int i = 0; i < 6; ++i)
      if (w[i] > 0.0f) j = i;
    if (kPhoton && wg > 0.0f) j = 6;
    if constexpr (kHvy) {
#pragma unroll
      for (int i = 0; i < kHeavy; ++i)
        if (wh[i] > 0.0f) j = 7 + i;
    }
  }
  if constexpr (kPhoton) {
    if (j == 6) {
      // photon: its share of the excitation from the spectrum, energy
      // (Mp^2 - Md^2) / (2 Mp) = eps (1 - eps / (2 Mp)) in the nucleus's rest
      // frame, isotropic, boosted to the lab
      const float sg = photon_sample_s(Yg, rng.next());
      const float eg = nu.E * sg * (2.0f - sg);
      const float Ed = nu.E * (1.0f - sg) * (1.0f - sg);
      const float Mp = row.M + nu.E;
      const float Eg = eg * (1.0f - 0.5f * eg / Mp);
      const float ct = 2.0f * rng.next() - 1.0f;
      const float st = sqrtf(fmaxf(0.0f, 1.0f - ct * ct));
      float sph, cph;
      sincospif(2.0f * rng.next(), &sph, &cph);
      const V3 qv = {Eg * st * cph, Eg * st * sph, Eg * ct};
      const V3 u = scale(1.0f / Mp, nu.P);
      const float uu = dot3(u, u);
      const float g = sqrtf(1.0f + uu);
      const float ig1 = 1.0f / (g + 1.0f);
      V3 pf;
      float Tf;
      boost_out(qv, 0.0f, u, g, ig1, uu * ig1, pf, Tf);
      em.on = true;
      em.kind = 6u | (1u << 8);
      em.T = sqrtf(dot3(pf, pf));
      em.u = unit(pf);
      nu.P = {nu.P.x - pf.x, nu.P.y - pf.y, nu.P.z - pf.z};
      nu.E = Ed;
      return false;
    }
  }
  float Uj = 0.0f, Vj = 0.0f, Yj = 0.0f, mj = 0.0f;
  int aj = 0, zj = 0;
#pragma unroll
  for (int i = 0; i < 6; ++i)
    if (i == j) {
      Uj = U[i];
      Vj = V[i];
      Yj = Y[i];
      mj = et.m[i];
      aj = fa[i];
      zj = fz[i];
    }
  if constexpr (kHvy) {
    if (j >= 7) {
      // the chosen heavier fragment's U, V and Y as its width had them
      const HeavyRow& hrow = bt.heavy[nu.A * bt.zstride + nu.Z];
#pragma unroll
      for (int i = 0; i < kHeavy; ++i)
        if (7 + i == j) {
          Vj = hrow.V[i];
          Uj = nu.E - hrow.S[i] - Vj;
          aj = ha[i];
          zj = hz[i];
          Yj = 2.0f * sqrtf((float)(nu.A - aj) * 0.125f * Uj);
          mj = bt.hmass[i];
        }
    }
  }
  const float s = spectrum_sample_s(Yj, rng.next());
  const float x = Uj * s * (2.0f - s);
  const float Ed = Uj * (1.0f - s) * (1.0f - s);
  const float eps = Vj + x;
  const int Ad = nu.A - aj, Zd = nu.Z - zj;
  const float Mp = row.M + nu.E;
  const float Mb = bt.chan[Ad * bt.zstride + Zd].M + Ed;
  const float inv2a = 0.5f / Mp;
  const float p2 = eps * (eps + 2.0f * mj) * ((eps + 2.0f * Mb) * inv2a) * ((eps + 2.0f * Mb + 2.0f * mj) * inv2a);
  const float ps = sqrtf(fmaxf(p2, 0.0f));
  const float ct = 2.0f * rng.next() - 1.0f;
  const float st = sqrtf(fmaxf(0.0f, 1.0f - ct * ct));
  float sph, cph;
  sincospif(2.0f * rng.next(), &sph, &cph);
  const V3 qv = {ps * st * cph, ps * st * sph, ps * ct};
  const V3 u = scale(1.0f / Mp, nu.P);
  const float uu = dot3(u, u);
  const float g = sqrtf(1.0f + uu);
  const float ig1 = 1.0f / (g + 1.0f);
  V3 pf;
  float Tf;
  boost_out(qv, mj, u, g, ig1, uu * ig1, pf, Tf);
  // the record's kinetic energy from the boosted momentum itself: the boost
  // form cancels for a fragment sent backward out of a moving nucleus, and a
  // heavy fragment left nearly at rest then has |p| = sqrt(T^2 + 2 T m)
  // badly determined by T; p^2 / (E + m) is accurate to a few ulps always
  {
    const float pf2 = dot3(pf, pf);
    Tf = pf2 / (sqrtf(pf2 + mj * mj) + mj);
  }
  em.on = true;
  em.kind = (uint32_t)j | (1u << 8);
  em.T = Tf;
  em.u = unit(pf);
  nu.P = {nu.P.x - pf.x, nu.P.y - pf.y, nu.P.z - pf.z};
  nu.A = Ad;
  nu.Z = Zd;
  nu.E = Ed;
  return false;
}

}  // namespace incdev
