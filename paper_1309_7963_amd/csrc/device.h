// device.h — device-side building blocks of the gfx950 cascade + evaporation
// kernels (arXiv:1309.7963, Sec. 2 and 3).  Everything here is FP32 IEEE
// arithmetic (Sec. 3.1 computes in single precision) except the binding-energy
// differences of the evaporation, which come from a double table so that no
// nuclear total energy is ever formed in FP32.
#pragma once

#include <stddef.h>

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/inc.h"

namespace incdev {

constexpr int kShells = 15;
constexpr int kMaxTargets = 16;
constexpr int kStackDepth = 64;      // LIFO guard (depth 64)
constexpr int kStackLdsMax = 4;      // stack entries per lane that may sit in LDS
constexpr int kMaxSegments = 10000;  // flight-segment guard per event
constexpr int kXsNodes = 512;        // log-spaced p_lab nodes
constexpr float kPi = 3.14159265358979323846f;
constexpr float kMassN = 939.565420f;
constexpr float kMassP = 938.272088f;
constexpr float kE2 = 1.44f;         // e^2, MeV fm
constexpr float kMbToFm2 = 0.1f;
constexpr float kPlo = 0.1374f;      // GeV/c; NN argument floor (T_lab ~ 10 MeV)
constexpr float kPhi = 1.5f;         // GeV/c; NN argument ceiling

constexpr uint16_t kFlagStack = 1, kFlagSegments = 2, kFlagEmpty = 4, kFlagRange = 0x8000;
// hand-over only (never in a residual): the residual is already written
constexpr uint16_t kMidFinal = 0x4000;

// --------------------------------------------------------------- tables
// One target nucleus: 15 shells (Sec. 2.2).  Index [species][shell], species
// 0 = neutron, 1 = proton; r2[i] = (i R / 15)^2 for i = 0..15.
struct NucTab {
  float r2[16];
  float rho[2][16];  // fm^-3
  float pF[2][16];   // MeV/c
  float EF[2][16];   // MeV
  float R, EB, EC;
  float EFmin[2];    // smallest E_F per species (outermost shell)
  float pFmax[2];    // largest p_F per species (innermost shell)
  int A, Z;
  float EYmax[2];    // total energy of a nucleon at pFmax, sqrt(pFmax^2 + m^2)
  float pad[5];
};
static_assert(sizeof(NucTab) % 16 == 0, "NucTab must stay 16-byte aligned");

// NN elastic table on a log grid of p_lab in [kPlo, kPhi] (Sec. 2.3, 3.1):
// columns [like] = sigma (mb), sigma_hat suffix maximum (mb), slope b
// ((GeV/c)^-2); like = 1 for pp/nn, 0 for np/pn.
struct XsTab {
  float sig[2][kXsNodes];
  float hat[2][kXsNodes];
  float slope[2][kXsNodes];
};
// The part of XsTab the event kernels stage in LDS: the cross-sections and
// their majorant.  The kernels take the slope b from its closed form
// (slope_b): linear interpolation across the unlike-pair breaks of b (0.225
// and 0.6 GeV/c, where 200 MeV collisions sit) errs by up to ~1e-3 and moves
// the sampled scattering angle; the closed form costs a few instructions per
// collision and frees 4 KB of LDS per block.  The slope columns stay in the
// device table for read-back.
struct XsLds {
  float sig[2][kXsNodes];
  float hat[2][kXsNodes];
};
static_assert(offsetof(XsTab, slope) == sizeof(XsLds), "XsLds is the head of XsTab");
// The same columns as node pairs: entry k of a column holds (v[k], v[k+1]),
// so an interpolation takes one 8-byte LDS read instead of two 4-byte ones,
// for twice the LDS (the launch-policy option table_layout = 1).
struct XsPairs {
  float2 sig[2][kXsNodes];
  float2 hat[2][kXsNodes];
};

// Evaporation constants (Sec. 2.4): fragment masses, mass numbers, charges,
// spin factors, a^(1/3), binding energies.
struct EvapTab {
  float m[6];
  float a13[6];
  float lngm[6];   // ln(g_j m_j)
  double B[6];
};

// Per mass number A = 0..kMaxA: A^(1/3) and ln A (evaporation geometry).
constexpr int kMaxA = 255;
struct MassTab {
  float a13[kMaxA + 1];
  float lnA[kMaxA + 1];
};

// Per-call constants shared by the kernels.
struct Opts {
  int no_pauli, no_evaporation, stop_after_first;
  float const_sigma_mb;  // > 0 overrides every NN cross-section
  float fixed_b;         // >= 0 fixes the impact parameter
  int evap_threshold, tent_threshold, kin_threshold, start_threshold;
  int same_stream;       // every event uses its segment's first id
};
// The test hooks of Opts (fixed impact parameter, constant cross-section, no
// Pauli blocking, stop after the first collision) at their neutral values, as
// compile-time constants: the kernels of contexts that set none of them are
// instantiated with this type, so that they hold none of the hooks' code or
// registers.
struct NoHooks {
  static constexpr float fixed_b = -1.0f;
  static constexpr float const_sigma_mb = 0.0f;
  static constexpr int no_pauli = 0;
  static constexpr int stop_after_first = 0;
};

// Evaporation constants of one nucleus (A, Z) (Sec. 2.4), computed once per
// context from the binding table: per channel j the separation energy S_j
// (+inf when the daughter does not exist), the Coulomb barrier V_j and
// ln(g_j m_j) + ln R_j^2; the nuclear mass M(A, Z); and for the optional
// photon channel ln(s0 / pi), s0 the slope of the photoabsorption
// cross-section (-inf: no dipole strength, N Z = 0).
struct ChanRow {
  float S[6], V[6], P[6];
  float M, lg;
};
static_assert(sizeof(ChanRow) == 80, "ChanRow layout");

// Heavier evaporation fragments (option, reading R20): the stable isotopes of
// Li to Mg, species 7 .. 6 + kHeavy, with ground-state multiplicities 2s + 1.
constexpr int kHeavy = 20;
#define INC_HEAVY_A {6, 7, 9, 10, 11, 12, 13, 14, 15, 16, 17, 18, 19, 20, 21, 22, 23, 24, 25, 26}
#define INC_HEAVY_Z {3, 3, 4, 5, 5, 6, 6, 7, 7, 8, 8, 8, 9, 10, 10, 10, 11, 12, 12, 12}
#define INC_HEAVY_G {3, 4, 4, 7, 4, 1, 2, 3, 2, 1, 6, 1, 2, 1, 4, 1, 4, 1, 6, 1}
// Per (A, Z): the heavier channels' S_j (+inf for a missing daughter), V_j and
// ln(g_j m_j R_j^2), as ChanRow holds them for the particles.
struct HeavyRow {
  float S[kHeavy], V[kHeavy], P[kHeavy];
};

// Binding energies B(A, Z) in double and the evaporation rows, for A <= amax,
// Z <= zmax (row of (A, Z) at A * zstride + Z).
struct BindTab {
  const double* B;
  int zstride;  // zmax + 1
  int amax, zmax;
  const ChanRow* chan;
  const HeavyRow* heavy;  // option heavy_fragments (NULL when off)
  const float* hmass;     // the heavier fragments' masses (kHeavy)
};

// --------------------------------------------------------------- Philox
// a ^ b ^ k in one instruction: v_bitop3_b32 with truth table 0x96 (odd
// parity of the three inputs).  k is wave-uniform (a round key).
__device__ __forceinline__ uint32_t xor3_uniform(uint32_t a, uint32_t b, uint32_t k) {
  uint32_t r;
  asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(r) : "v"(a), "v"(b), "s"(k));
  return r;
}

// Philox4x32-10 (Salmon et al., SC'11).  The key must be wave-uniform.
__device__ __forceinline__ void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                              uint32_t k0, uint32_t k1, uint32_t out[4]) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    // one 32 x 32 -> 64-bit multiply gives both halves of each product
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = xor3_uniform(hi1, c1, k0);
    const uint32_t n2 = xor3_uniform(hi0, c3, k1);
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

// Per-event stream: key = seed, counter = (block, id lo, id hi, 0); the four
// words of a block are used in order; u = ((w >> 9) + 1/2) 2^-23, exact in
// FP32 and strictly inside (0, 1).
//
// Two blocks are buffered (a: current, b: next).  Every step calls ensure(k)
// once at its start with the most words it can draw, so the Philox rounds run
// with all lanes of that step together instead of at scattered draw sites;
// next() generates only the rare word the two blocks could not hold.  The
// order of the words is the stream order whatever the buffering.
//
// The key is the launch's seed, set once before any event starts and never
// changed, so it stays wave-uniform: the key schedule runs on the scalar unit
// and only the counter arithmetic takes vector instructions.
struct Rng {
  uint32_t k0, k1, id0, id1;
  uint32_t blk;    // next block to generate
  uint32_t a[4], b[4];
  uint32_t pos;    // next word of a (4 = a used up)
  uint32_t nb;     // words valid in b (0 or 4)

  __device__ __forceinline__ void set_key(uint64_t seed) {
    k0 = (uint32_t)seed;
    k1 = (uint32_t)(seed >> 32);
  }
  __device__ __forceinline__ void init(uint64_t id) {
    id0 = (uint32_t)id;
    id1 = (uint32_t)(id >> 32);
    blk = 0;
    pos = 4;
    nb = 0;
  }
  __device__ __forceinline__ void gen(uint32_t out[4]) {
    philox4x32_10(blk, id0, id1, 0u, k0, k1, out);
    ++blk;
  }
  __device__ __forceinline__ uint32_t avail() const { return 4u - pos + nb; }
  __device__ __forceinline__ void shift() {
    a[0] = b[0];
    a[1] = b[1];
    a[2] = b[2];
    a[3] = b[3];
    pos = 0;
    nb = 0;
  }
  // Prefetch so that at least k words are buffered when the two blocks can
  // hold them (always for k <= 5); next() generates any word still missing.
  // One generation site per round, whichever block it fills, so lanes that
  // refill a and lanes that refill b share one pass of the Philox rounds.
  __device__ __forceinline__ void ensure(uint32_t k) {
    if (pos == 4 && nb == 4) shift();
    if (avail() < k && (pos == 4 || nb == 0)) {
      uint32_t w[4];
      gen(w);
      if (pos == 4) {
        a[0] = w[0]; a[1] = w[1]; a[2] = w[2]; a[3] = w[3];
        pos = 0;
      } else {
        b[0] = w[0]; b[1] = w[1]; b[2] = w[2]; b[3] = w[3];
        nb = 4;
      }
    }
    if (avail() < k && nb == 0) {
      gen(b);
      nb = 4;
    }
  }
  // Resume after `drawn` uniforms.
  __device__ __forceinline__ void seek(uint32_t drawn) {
    blk = drawn >> 2;
    pos = drawn & 3u;
    nb = 0;
    if (pos) gen(a);
    else pos = 4;
  }
  __device__ __forceinline__ uint32_t drawn() const { return blk * 4u - avail(); }
  // Next uniform of the stream.
  __device__ __forceinline__ float next() {
    if (pos >= 4) {
      if (nb) {
        shift();
      } else {
        gen(a);
        pos = 0;
      }
    }
    const uint32_t v = pos == 0 ? a[0] : pos == 1 ? a[1] : pos == 2 ? a[2] : a[3];
    ++pos;
    return (float)(v >> 9) * 0x1p-23f + 0x1p-24f;
  }
};

// ------------------------------------------------------------ small math
__device__ __forceinline__ float nucleon_mass(int sp) { return sp ? kMassP : kMassN; }

// log(1 + x) for x > -1 from logf (Goldberg, "What every computer scientist
// should know about floating-point arithmetic", 1991, Theorem 4): with
// u = fl(1 + x), log(1 + x) = log(u) x / (u - 1), and x itself when u == 1.
// A few ulp, at the cost of one logf and one division.
__device__ __forceinline__ float log1p_acc(float x) {
  const float u = 1.0f + x;
  return u == 1.0f ? x : logf(u) * (x / (u - 1.0f));
}
__device__ __forceinline__ float kinetic_of(float p, float m) { return p * p / (sqrtf(p * p + m * m) + m); }

struct V3 {
  float x, y, z;
};
__device__ __forceinline__ float dot3(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ V3 axpy(float s, V3 a, V3 b) { return {s * a.x + b.x, s * a.y + b.y, s * a.z + b.z}; }
__device__ __forceinline__ V3 scale(float s, V3 a) { return {s * a.x, s * a.y, s * a.z}; }
__device__ __forceinline__ V3 unit(V3 a) { return scale(rsqrtf(dot3(a, a)), a); }

// Unit vector at polar angle (cos c, sin s) and azimuth 2 pi u_phi from a.
__device__ __forceinline__ V3 rotate(V3 a, float c, float s, float u_phi) {
  float sp, cp;
  sincospif(2.0f * u_phi, &sp, &cp);
  const float st = sqrtf(a.x * a.x + a.y * a.y);
  if (st > 1e-6f) {
    const float inv = 1.0f / st;
    const V3 e1 = {a.x * a.z * inv, a.y * a.z * inv, -st};
    const V3 e2 = {-a.y * inv, a.x * inv, 0.0f};
    return {c * a.x + s * (cp * e1.x + sp * e2.x), c * a.y + s * (cp * e1.y + sp * e2.y),
            c * a.z + s * (cp * e1.z + sp * e2.z)};
  }
  return {s * cp, s * sp, a.z >= 0.0f ? c : -c};
}

// Boost a momentum q of mass m from a frame with gamma*beta = u, gamma = g;
// ig1 = 1 / (g + 1) and uu1 = (u.u) / (g + 1) are shared by the products of
// one decay.  T = (gamma - 1) m + gamma T* + u.q without forming total energies.
__device__ __forceinline__ void boost_out(V3 q, float m, V3 u, float g, float ig1, float uu1, V3& p, float& T) {
  const float q2 = dot3(q, q);
  const float E = sqrtf(q2 + m * m);
  const float uq = dot3(u, q);
  p = axpy(uq * ig1 + E, u, q);
  T = g * (q2 / (E + m)) + uu1 * m + uq;
}
__device__ __forceinline__ float inv_nucleon_mass(int sp) { return sp ? 1.0f / kMassP : 1.0f / kMassN; }

// -------------------------------------------------------- cross-sections
// Table coordinate of p_lab: nodes are equally spaced in log p between kPlo and
// kPhi; the hardware log2 (about 1 ulp) places p between two nodes.
__device__ __forceinline__ void xs_coord(float p_GeV, int& k, float& f) {
  const float pc = fminf(fmaxf(p_GeV, kPlo), kPhi);
  const float scale = (float)(kXsNodes - 1) / 3.4485086f;  // log2(kPhi / kPlo)
  float x = __builtin_amdgcn_logf(pc * (1.0f / kPlo)) * scale;
  x = fminf(fmaxf(x, 0.0f), (float)(kXsNodes - 1));
  k = min((int)x, kXsNodes - 2);
  f = x - (float)k;
}
// Slope b ((GeV/c)^-2) of the CM angular distribution exp(b t) (Sec. 2.3,
// reading R9) at p_lab (GeV/c, clamped to the table's range like the
// cross-sections): like pairs 5.5 p^8 / (7.7 + p^8); unlike pairs 0 below
// 0.225, 16.53 (p - 0.225) below 0.6, -1.63 p + 7.16 above.
__device__ __forceinline__ float slope_b(int like, float p_GeV) {
  const float p = fminf(fmaxf(p_GeV, kPlo), kPhi);
  const float p2 = p * p, p4 = p2 * p2, p8 = p4 * p4;
  const float bl = 5.5f * p8 / (7.7f + p8);
  const float bu = p < 0.225f ? 0.0f : (p < 0.6f ? 16.53f * (p - 0.225f) : 7.16f - 1.63f * p);
  return like ? bl : bu;
}
__device__ __forceinline__ float xs_lerp(const float* col, int k, float f);
// sigma and its majorant of like (1) / unlike (0) pairs at table coordinate
// (k, f), from either LDS layout (the same arithmetic, the same result)
__device__ __forceinline__ float xs_sig(const XsLds& xs, int like, int k, float f) { return xs_lerp(xs.sig[like], k, f); }
__device__ __forceinline__ float xs_hat(const XsLds& xs, int like, int k, float f) { return xs_lerp(xs.hat[like], k, f); }
__device__ __forceinline__ float xs_sig(const XsPairs& xs, int like, int k, float f) {
  const float2 v = xs.sig[like][k];
  return v.x + f * (v.y - v.x);
}
__device__ __forceinline__ float xs_hat(const XsPairs& xs, int like, int k, float f) {
  const float2 v = xs.hat[like][k];
  return v.x + f * (v.y - v.x);
}
__device__ __forceinline__ float xs_lerp(const float* col, int k, float f) {
  const float a = col[k], b = col[k + 1];
  return a + f * (b - a);
}

// Majorant flight cross-sections (fm^2) for a particle of species sp with
// excess energy eps: smallest own momentum (at the smallest E_F) against the
// largest Fermi momentum of each target species.
template <class XS, class O>
__device__ __forceinline__ void majorant(const NucTab& nt, const XS& xs, const O& o, int sp, float eps,
                                         float& sh0, float& sh1) {
  const float mx = nucleon_mass(sp);
  const float T = eps + nt.EFmin[sp];
  const float p = sqrtf(T * T + 2.0f * T * mx);
  const float Ex = T + mx;
  float sh[2];
#pragma unroll
  for (int y = 0; y < 2; ++y) {
    const float pF = nt.pFmax[y];
    const float pmin = fmaxf(0.0f, (p * nt.EYmax[y] - Ex * pF) * inv_nucleon_mass(y)) * 1e-3f;
    float s;
    if (o.const_sigma_mb > 0.0f) {
      s = o.const_sigma_mb;
    } else {
      int k;
      float f;
      xs_coord(pmin, k, f);
      s = xs_hat(xs, sp == y, k, f);
    }
    sh[y] = s * kMbToFm2;
  }
  sh0 = sh[0];
  sh1 = sh[1];
}

// Classical refraction at a potential step (reading of Chen et al., Sec. 2.3):
// tangential momentum kept, T - V conserved, reflection when the normal
// component cannot be formed.  Returns true when transmitted.
__device__ __forceinline__ bool refract(V3& d, V3 n, float T_from, float T_to, float m) {
  const float p_from = sqrtf(T_from * T_from + 2.0f * T_from * m);
  const float dn = dot3(d, n);
  const float pn = p_from * dn;
  if (T_to > 0.0f) {
    const float pn2 = pn * pn + (T_to - T_from) * (T_to + T_from + 2.0f * m);
    if (pn2 > 0.0f) {
      const float pnn = copysignf(sqrtf(pn2), pn);
      const V3 q = {p_from * d.x + (pnn - pn) * n.x, p_from * d.y + (pnn - pn) * n.y,
                    p_from * d.z + (pnn - pn) * n.z};
      d = unit(q);
      return true;
    }
  }
  d = axpy(-2.0f * dn, n, d);
  return false;
}

// ------------------------------------------------------------ evaporation
// ln I(a, U), I = int_0^U x exp(2 sqrt(a (U - x))) dx
//   = [e^Y (2Y^2 - 6Y + 6) + Y^2 - 6] / (8 a^2),  Y = 2 sqrt(a U),
// with the all-positive series (1/4a^2) sum_{n>=4} (n-1)(n-3) Y^n/n! below Y = 2.
// a = A_d / 8, so ln(8 a^2) = 2 ln A_d - ln 8 and ln(4 a^2) = 2 ln A_d - ln 16.
__device__ __forceinline__ float log_width_integral(float Y, float lnAd) {
  if (Y < 2.0f) {
    float term = Y * Y * Y * Y * (1.0f / 24.0f);
    float sum = 0.0f;
#pragma unroll
    for (int n = 4; n < 22; ++n) {
      sum += (float)((n - 1) * (n - 3)) * term;
      term *= Y * (1.0f / (float)(n + 1));  // unrolled: a constant reciprocal, no division
    }
    return logf(sum) - (2.0f * lnAd - 2.7725887f);
  }
  const float k = (2.0f * Y - 6.0f) * Y + 6.0f + expf(-Y) * (Y * Y - 6.0f);
  return Y + logf(k) - (2.0f * lnAd - 2.0794415f);
}

// Kinetic-energy excess x in [0, U] with density ~ x exp(2 sqrt(a (U - x))).
// With Y = 2 sqrt(a U), t = Y - 2 sqrt(a (U - x)) and s = t / Y in [0, 1]:
// x = U s (2 - s), U - x = U (1 - s)^2, and the CDF in s is K(s) / K(1) with
// dK/ds = k(s) = s (2 - s) (1 - s) e^{-Y s} (times Y^4 for Y >= 1, the scale
// of the closed form).  The sampler solves on the lower half of the CDF
// (u <= 1/2) with K(s) and on the upper half with the tail mass K(1) - K(s),
// each from a form without cancellation: K by its series in s while Y s < 1
// for lower-tail targets (u < 0.01; always for Y < 1), else closed form; the
// tail mass in closed form (Y >= 1).  The root is found by bracketed Newton
// iteration to a residual of 1e-5 of the target mass or a relative step of
// 1e-6, so tail samples keep their relative accuracy.  For large Y the start is the quantile of the Gamma(2) limit,
// x = Y s with 1 - u = (1 + x) e^{-x}, from one fixed-point step.
__device__ __forceinline__ float spectrum_series(float Y, float s) {
  // sum_m (-Y)^m / m! [2 s^{m+2}/(m+2) - 3 s^{m+3}/(m+3) + s^{m+4}/(m+4)]
  float c = 1.0f, sm = s * s, sum = 0.0f;
#pragma unroll
  for (int m = 0; m < 12; ++m) {
    // unrolled: the coefficients are constant reciprocals, no division
    sum += c * sm * (2.0f / (float)(m + 2) - s * (3.0f / (float)(m + 3)) + s * s * (1.0f / (float)(m + 4)));
    c *= -Y * (1.0f / (float)(m + 1));
    sm *= s;
  }
  return sum;
}
// e^{-t} Q(t) with t = Y s: the closed form K(s) = Q(0) - e^{-t} Q(t) (Y >= 1)
__device__ __forceinline__ float spectrum_eQ(float Y, float t) {
  const float Q = 2.0f * Y * Y * (1.0f + t) - 3.0f * Y * ((t + 2.0f) * t + 2.0f) + ((t + 3.0f) * t + 6.0f) * t + 6.0f;
  return expf(-t) * Q;
}
// K(s); `deep`: a lower-tail target (u < 0.01), where the closed form's
// cancellation would show, so the series is taken while Y s < 1
__device__ __forceinline__ float spectrum_K(float Y, float s, bool deep = false) {
  if (Y < 1.0f) return spectrum_series(Y, s);
  if (deep && Y * s < 1.0f) {
    const float Y2 = Y * Y;
    return Y2 * Y2 * spectrum_series(Y, s);
  }
  return ((2.0f * Y - 6.0f) * Y + 6.0f) - spectrum_eQ(Y, Y * s);
}
// K(1) - K(s), the CDF's upper tail mass
__device__ __forceinline__ float spectrum_Kc(float Y, float s, float K1) {
  if (Y < 1.0f) return K1 - spectrum_series(Y, s);
  return spectrum_eQ(Y, Y * s) - spectrum_eQ(Y, Y);
}
__device__ __forceinline__ float spectrum_dK(float Y, float s) {
  const float core = s * (2.0f - s) * (1.0f - s) * expf(-Y * s);
  if (Y < 1.0f) return core;
  const float Y2 = Y * Y;
  return Y2 * Y2 * core;
}
__device__ __forceinline__ float spectrum_sample_s(float Y, float u) {
  const float K1 = spectrum_K(Y, 1.0f);
  const bool upper = u > 0.5f;
  // lower half: K(s) = u K1, increasing in s; upper half: K1 - K(s) = (1 - u) K1
  const float target = (upper ? 1.0f - u : u) * K1;
  const float ftol = 1e-5f * target;
  const bool deep = u < 0.01f;
  float lo = 0.0f, hi = 1.0f;
  float s = 0.5f;
  if (Y > 4.0f) {
    const float x0 = -log1p_acc(-u);
    s = fminf(fmaxf((x0 + log1p_acc(x0)) / Y, 1e-4f), 0.95f);
  }
  for (int it = 0; it < 40; ++it) {
    // F increases with s on both halves
    const float F = upper ? target - spectrum_Kc(Y, s, K1) : spectrum_K(Y, s, deep) - target;
    if (F < 0.0f) lo = s; else hi = s;
    if (fabsf(F) <= ftol) break;
    const float dF = spectrum_dK(Y, s);
    float sn = (dF > 0.0f) ? s - F / dF : 0.5f * (lo + hi);
    if (!(sn > lo && sn < hi)) sn = 0.5f * (lo + hi);
    const float step = fabsf(sn - s);
    s = sn;
    if (step <= 1e-6f * s || hi - lo <= 1e-6f * hi) break;
  }
  return fminf(fmaxf(s, 0.0f), 1.0f);
}

// ------------------------------------------------------------ photon channel
// Optional (off by default; Sec. 2 has de-excitation by particles, then
// photons, and Sec. 2.4 leaves photons out).  Width from detailed balance
// with a photoabsorption cross-section s0 eps (rising to the giant-dipole
// energy, holding the classical dipole sum), in the particle widths' units:
// w = (s0/pi) J, J = int_0^E eps^3 exp(2 sqrt(a (E - eps))) d eps, a = A/8.
// With Y = 2 sqrt(a E) and eps = E s (2 - s): J = 2 E^4 e^Y Kg(Y, 1),
// Kg(Y, s) = int_0^s q(t) e^{-Y t} dt, q(t) = t^3 (2 - t)^3 (1 - t)
// = 8 t^3 - 20 t^4 + 18 t^5 - 7 t^6 + t^7; the CDF of s is Kg(Y, s) / Kg(Y, 1).
constexpr float kPhotonMin = 0.1f;  // MeV: the channel is open above this
__device__ __forceinline__ float photon_q(float t) {
  return t * t * t * ((((t - 7.0f) * t + 18.0f) * t - 20.0f) * t + 8.0f);
}
__device__ __forceinline__ float photon_series(float Y, float s) {
  // sum_m (-Y)^m / m! int_0^s q(t) t^m dt (converges for Y s < 4 in 21 terms)
  float c = 1.0f, sm = s * s * s * s, sum = 0.0f;
#pragma unroll
  for (int m = 0; m < 21; ++m) {
    sum += c * sm *
           (8.0f / (float)(m + 4) -
            s * (20.0f / (float)(m + 5) -
                 s * (18.0f / (float)(m + 6) - s * (7.0f / (float)(m + 7) - s * (1.0f / (float)(m + 8))))));
    c *= -Y * (1.0f / (float)(m + 1));
    sm *= s;
  }
  return sum;
}
// S(t) = sum_j q^(j)(t) / Y^(j+1) as a polynomial in t (c7 = 1/Y,
// c_n = (q_n + (n + 1) c_{n+1}) / Y), so that int q e^{-Y t} = -e^{-Y t} S(t);
// returns S(t) and S(0) = c0
__device__ __forceinline__ float photon_S(float Y, float t, float& c0) {
  const float iy = 1.0f / Y;
  const float c7 = iy;
  const float c6 = (-7.0f + 7.0f * c7) * iy;
  const float c5 = (18.0f + 6.0f * c6) * iy;
  const float c4 = (-20.0f + 5.0f * c5) * iy;
  const float c3 = (8.0f + 4.0f * c4) * iy;
  const float c2 = 3.0f * c3 * iy;
  const float c1 = 2.0f * c2 * iy;
  c0 = c1 * iy;
  return ((((((c7 * t + c6) * t + c5) * t + c4) * t + c3) * t + c2) * t + c1) * t + c0;
}
__device__ __forceinline__ float photon_K(float Y, float s) {
  if (Y < 4.0f || Y * s < 4.0f) return photon_series(Y, s);
  float c0;
  const float S = photon_S(Y, s, c0);
  return c0 - expf(-Y * s) * S;
}
// Kg(1) - Kg(s), the CDF's upper tail mass
__device__ __forceinline__ float photon_Kc(float Y, float s, float K1) {
  if (Y < 4.0f) return K1 - photon_series(Y, s);
  float c0;
  const float Ss = photon_S(Y, s, c0);
  const float S1 = photon_S(Y, 1.0f, c0);
  return expf(-Y * s) * Ss - expf(-Y) * S1;
}
// ln J(a, E) - ln 2: Y + 4 ln E + ln Kg(Y, 1)
__device__ __forceinline__ float log_photon_integral(float Y, float E) {
  return Y + 4.0f * logf(E) + logf(photon_K(Y, 1.0f)) + 0.6931472f;
}
// s of the photon's share eps = E s (2 - s) for a uniform u: on the lower
// half of the CDF the root of Kg(Y, s) = u Kg(Y, 1), on the upper half of
// Kg(Y, 1) - Kg(Y, s) = (1 - u) Kg(Y, 1), by bracketed Newton iteration (as
// the particles').
__device__ __forceinline__ float photon_sample_s(float Y, float u) {
  const float K1 = photon_K(Y, 1.0f);
  const bool upper = u > 0.5f;
  const float target = (upper ? 1.0f - u : u) * K1;
  const float ftol = 1e-5f * target;
  float lo = 0.0f, hi = 1.0f;
  // start near the median of the large-Y limit t^3 e^{-Y t} (Gamma(4))
  float s = fminf(0.5f, 3.672f / Y);
  for (int it = 0; it < 40; ++it) {
    const float F = upper ? target - photon_Kc(Y, s, K1) : photon_K(Y, s) - target;
    if (F < 0.0f) lo = s; else hi = s;
    if (fabsf(F) <= ftol) break;
    const float dF = photon_q(s) * expf(-Y * s);
    float sn = (dF > 0.0f) ? s - F / dF : 0.5f * (lo + hi);
    if (!(sn > lo && sn < hi)) sn = 0.5f * (lo + hi);
    const float step = fabsf(sn - s);
    s = sn;
    if (step <= 1e-6f * s || hi - lo <= 1e-6f * hi) break;
  }
  return fminf(fmaxf(s, 0.0f), 1.0f);
}

// ------------------------------------------------------------- writer
// Wave-compacted writer (Sec. 3.3 writes evaporated particles uncoalesced):
// lanes that emit a record this iteration append it to the wave's LDS buffer
// at (fill + rank among emitting lanes); when the buffer could overflow, the
// wave reserves space with one global atomic and all 64 lanes copy the
// buffer out contiguously into the SoA arrays.
constexpr int kWriterCap = 128;      // records per wave buffer (cascade kernels)
constexpr int kWriterCapEvap = 256;  // records per wave buffer (evaporation kernels)
constexpr int kRecWords = 6;     // event, species | stage << 8 | segment << 16, T, ux, uy, uz
// One append adds up to a record per lane after at most one flush, so a wave's
// buffer must hold a full wave of records (a smaller one would overflow into
// the next wave's LDS).
static_assert(kWriterCap >= 64 && kWriterCapEvap >= 64, "writer buffer below one wave of records");

// One segment of a launch: a request with its own event ids and output
// buffers (all segments of a launch share the launch's random-stream key).
// Event i of the launch with start <= i < start + n belongs to the segment,
// has id first_id + (i - start) and writes its residual to res[i - start] and
// its secondaries to the segment's arrays (records hold i - start).
// counters: [0] secondaries produced, [1] flagged.
struct Segment {
  uint32_t start, n;
  uint64_t first_id;
  inc_residual* res;
  uint32_t* ev;
  uint8_t* species;
  uint8_t* stage;
  float* T;
  float* ux;
  float* uy;
  float* uz;
  unsigned long long cap;
  unsigned long long* counters;
  uint32_t* hist;  // optional history words, 2 per event (NULL: not written)
};

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint32_t rank_in(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Segment holding launch event i (segments are sorted by start).
__device__ __forceinline__ int segment_of(const Segment* segs, int n_seg, uint32_t i) {
  int lo = 0, hi = n_seg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (segs[mid].start <= i) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Ring output (streaming mode).  Host placement: records go to a ring of
// `mask + 1` slots in coherent host memory while a host thread drains it.  A
// wave reserves `fill` sequence numbers on the device counter `head`, waits
// (bounded) until the consumer's `tail` leaves room, writes the records'
// payload, then - after a system-scope release fence - their tags (sequence
// number + 1).  The consumer takes slot s & mask once its tag equals s + 1.
// Device placement (`done` set, `tag` NULL): the ring is in device memory
// (from `ev`; the other field pointers are unused) and is cut into chunks of
// 2^chunk_shift slots.  A wave writes its records with
// ordinary stores, makes them visible device-wide (agent-scope release), and
// adds their number to the counter of each chunk they fall in; the wave that
// completes a chunk clears its counter and publishes the chunk number + 1 in
// the host array `ready`, and the host copies the chunk out with an
// asynchronous copy.  The ring is a structure of arrays so that a wave's
// stores are contiguous (256 bytes per array and store instruction).
struct RingDev {
  uint32_t* tag;                    // host memory, one array per field; NULL = off
  uint32_t* ev;
  uint32_t* kind;
  uint32_t* T;                      // float bits
  uint32_t* ux;
  uint32_t* uy;
  uint32_t* uz;
  unsigned long long mask;          // slots - 1 (slots a power of two)
  unsigned long long* head;         // device counter: sequence numbers handed out
  const unsigned long long* tail;   // host memory: records consumed so far
  unsigned int* error;              // host memory: 1 = producer gave up waiting
  unsigned long long spin_limit;    // waits of ~1.7 us before giving up
  unsigned long long* done;         // device placement: records written per chunk (NULL: host placement)
  unsigned long long* ready;        // device placement, host memory: chunk number + 1 once complete
  unsigned long long chunk_mask;    // chunks in the ring - 1
  unsigned int chunk_shift;         // log2 of the slots per chunk
};

__device__ __forceinline__ void sys_store(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Device placement.  Must be called by all lanes of the wave.
__device__ __forceinline__ void ring_flush_device(const uint32_t* buf, int fill, const RingDev& R) {
  unsigned long long base = 0;
  int ok = 1;
  if (lane_id() == 0) {
    base = atomicAdd(R.head, (unsigned long long)fill);
    unsigned long long t = __hip_atomic_load(R.tail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    unsigned long long spins = 0;
    while (base + (unsigned long long)fill > t + R.mask + 1ull) {
      if (++spins > R.spin_limit ||
          __hip_atomic_load(R.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) != 0u) {
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(63);
      t = __hip_atomic_load(R.tail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
    if (!ok) __hip_atomic_fetch_or(R.error, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  }
  base = __shfl(base, 0);
  ok = __shfl(ok, 0);
  if (!ok) return;
  // chunk-major layout: chunk q holds its six fields one after another
  // (6 x 2^chunk_shift words from R.ev + 6 q 2^chunk_shift), so a complete
  // chunk leaves in one copy
  const unsigned long long per = 1ull << R.chunk_shift;
  for (int i = lane_id(); i < fill; i += 64) {
    const unsigned long long k = (base + (unsigned long long)i) & R.mask;
    const uint32_t* r = buf + i * kRecWords;
    uint32_t* d = R.ev + (k >> R.chunk_shift) * 6ull * per + (k & (per - 1ull));
    d[0] = r[0];
    d[per] = r[1];
    d[2 * per] = r[2];
    d[3 * per] = r[3];
    d[4 * per] = r[4];
    d[5 * per] = r[5];
  }
  // the records reach device memory (past this XCD's L2) before they count
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  if (lane_id() == 0) {
    const unsigned long long end = base + (unsigned long long)fill;
    for (unsigned long long c = base >> R.chunk_shift; c <= (end - 1ull) >> R.chunk_shift; ++c) {
      const unsigned long long lo = c << R.chunk_shift;
      const unsigned long long n = min(end, lo + per) - max(base, lo);
      unsigned long long* cnt = R.done + (c & R.chunk_mask);
      const unsigned long long old = __hip_atomic_fetch_add(cnt, n, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
      if (old + n == per) {
        // the chunk is complete: its counter starts over for the next lap,
        // and the host learns the chunk number
        __hip_atomic_store(cnt, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
        __hip_atomic_store(R.ready + (c & R.chunk_mask), c + 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      }
    }
  }
}

// Must be called by all lanes of the wave.
__device__ __forceinline__ void ring_flush(const uint32_t* buf, int fill, const RingDev& R) {
  unsigned long long base = 0;
  int ok = 1;
  if (lane_id() == 0) {
    base = atomicAdd(R.head, (unsigned long long)fill);
    unsigned long long t = __hip_atomic_load(R.tail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    unsigned long long spins = 0;
    while (base + (unsigned long long)fill > t + R.mask + 1ull) {
      if (++spins > R.spin_limit ||
          __hip_atomic_load(R.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) != 0u) {
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(63);
      t = __hip_atomic_load(R.tail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
    if (!ok) __hip_atomic_fetch_or(R.error, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  }
  base = __shfl(base, 0);
  ok = __shfl(ok, 0);
  if (!ok) return;
  for (int i = lane_id(); i < fill; i += 64) {
    const unsigned long long k = (base + (unsigned long long)i) & R.mask;
    const uint32_t* r = buf + i * kRecWords;
    sys_store(R.ev + k, r[0]);
    sys_store(R.kind + k, r[1]);
    sys_store(R.T + k, r[2]);
    sys_store(R.ux + k, r[3]);
    sys_store(R.uy + k, r[4]);
    sys_store(R.uz + k, r[5]);
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
  for (int i = lane_id(); i < fill; i += 64) {
    const unsigned long long k = (base + (unsigned long long)i) & R.mask;
    sys_store(R.tag + k, (uint32_t)(base + (unsigned long long)i + 1ull));
  }
}

// Must be called by all lanes of the wave.  The wave's records are copied out
// 64 at a time; within a group of 64 the lanes of each distinct segment
// reserve their slots with one atomic and store contiguously.  kRing: the
// records go to the ring of `ring` instead (a separate instantiation of the
// kernels, so that the others hold none of the ring's code and registers).
template <bool kRing>
__device__ __forceinline__ void writer_flush(uint32_t* buf, int& fill, const Segment* segs, const RingDev& ring) {
  if (fill == 0) return;
  __builtin_amdgcn_wave_barrier();
  if constexpr (kRing) {
    if (ring.done)
      ring_flush_device(buf, fill, ring);
    else
      ring_flush(buf, fill, ring);
    __builtin_amdgcn_wave_barrier();
    fill = 0;
    return;
  }
  // Usual case: every record of the buffer belongs to one segment, which
  // reserves all of them with one atomic.
  const int seg_first = (int)(buf[1] >> 16);
  bool mixed = false;
  for (int i = lane_id(); i < fill; i += 64) mixed |= (int)(buf[i * kRecWords + 1] >> 16) != seg_first;
  if (!__any(mixed)) {
    unsigned long long base = 0;
    if (lane_id() == 0) base = atomicAdd(&segs[seg_first].counters[0], (unsigned long long)fill);
    const Segment& S = segs[seg_first];
    base = __shfl(base, 0);
    for (int i = lane_id(); i < fill; i += 64) {
      const uint32_t* r = buf + i * kRecWords;
      const unsigned long long k = base + (unsigned long long)i;
      if (k < S.cap) {
        S.ev[k] = r[0];
        S.species[k] = (uint8_t)(r[1] & 0xFFu);
        S.stage[k] = (uint8_t)((r[1] >> 8) & 0xFFu);
        S.T[k] = __uint_as_float(r[2]);
        S.ux[k] = __uint_as_float(r[3]);
        S.uy[k] = __uint_as_float(r[4]);
        S.uz[k] = __uint_as_float(r[5]);
      }
    }
    __builtin_amdgcn_wave_barrier();
    fill = 0;
    return;
  }
  for (int g = 0; g < fill; g += 64) {
    const int i = g + lane_id();
    const bool have = i < fill;
    const uint32_t* r = buf + (have ? i : 0) * kRecWords;
    const int seg = have ? (int)(r[1] >> 16) : -1;
    uint64_t todo = __ballot(have);
    while (todo) {
      const int lead = __ffsll((unsigned long long)todo) - 1;
      const int s0 = __shfl(seg, lead);
      const uint64_t m = __ballot(have && seg == s0);
      unsigned long long base = 0;
      if (lane_id() == lead) base = atomicAdd(&segs[s0].counters[0], (unsigned long long)__popcll(m));
      base = __shfl(base, lead);
      if (have && seg == s0) {
        const Segment& S = segs[s0];
        const unsigned long long k = base + rank_in(m);
        if (k < S.cap) {
          S.ev[k] = r[0];
          S.species[k] = (uint8_t)(r[1] & 0xFFu);
          S.stage[k] = (uint8_t)((r[1] >> 8) & 0xFFu);
          S.T[k] = __uint_as_float(r[2]);
          S.ux[k] = __uint_as_float(r[3]);
          S.uy[k] = __uint_as_float(r[4]);
          S.uz[k] = __uint_as_float(r[5]);
        }
      }
      todo &= ~m;
    }
  }
  __builtin_amdgcn_wave_barrier();
  fill = 0;
}

// Must be called by all lanes of the wave.  ev: index of the event in its
// segment; kind: species | stage << 8 | segment << 16.  kCap: records the
// wave's buffer holds.
template <bool kRing, int kCap = kWriterCap>
__device__ __forceinline__ void writer_append(uint32_t* buf, int& fill, const Segment* segs, const RingDev& ring,
                                              bool emit, uint32_t ev, uint32_t kind, float T, V3 u) {
  const uint64_t m = __ballot(emit);
  if (m == 0) return;
  const int cnt = __popcll(m);
  if (fill + cnt > kCap) writer_flush<kRing>(buf, fill, segs, ring);
  if (emit) {
    uint32_t* r = buf + (fill + (int)rank_in(m)) * kRecWords;
    r[0] = ev;
    r[1] = kind;
    r[2] = __float_as_uint(T);
    r[3] = __float_as_uint(u.x);
    r[4] = __float_as_uint(u.y);
    r[5] = __float_as_uint(u.z);
  }
  fill += cnt;
}

}  // namespace incdev
