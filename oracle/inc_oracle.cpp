/*
 * inc_oracle.cpp — CPU oracle for the intranuclear cascade + evaporation
 * method of arXiv:1309.7963 (Wan Chan Tseung & Beltran).
 *
 * TEST INFRASTRUCTURE ONLY: a plain, slow, double-precision, scalar
 * implementation.  It is the yardstick the GPU library is checked against and
 * is loaded only by the tests, the smoke check and the CPU-baseline leg of the
 * benchmark.  It shares no code with the GPU path.
 *
 * Each function names the passage of the paper it follows.  Where the paper
 * is silent (constants of the NN parameterisation, refraction rule, mean free
 * path, evaporation widths) the frozen readings of the design notes are used;
 * every such place says "reading".
 */
#include "inc_oracle.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <thread>
#include <vector>

namespace {

/* ---------------------------------------------------------------- constants */
constexpr double kPi = 3.14159265358979323846;
constexpr double kHbarC = 197.3269804;      /* MeV fm                        */
constexpr double kMassN = 939.565420;       /* neutron (MeV)                 */
constexpr double kMassP = 938.272088;       /* proton (MeV)                  */
constexpr double kE2 = 1.44;                /* e^2 (MeV fm)                  */
constexpr double kMbToFm2 = 0.1;            /* 1 mb = 0.1 fm^2               */
constexpr double kPlo = 0.1374;             /* NN argument floor (GeV/c), T_lab ~ 10 MeV */
constexpr double kPhi = 1.5;                /* NN argument ceiling (GeV/c)   */

inline double nucleon_mass(int sp) { return sp == 1 ? kMassP : kMassN; }

/* ------------------------------------------------------------- Philox4x32-10
 * Counter-based generator of Salmon et al. (SC'11), 10 rounds.  The per-event
 * stream uses key = (seed lo, seed hi), counter = (block j, id lo, id hi, 0)
 * and consumes the four output words in order. */
void philox(const uint32_t c_in[4], const uint32_t k_in[2], uint32_t out[4]) {
  uint32_t c0 = c_in[0], c1 = c_in[1], c2 = c_in[2], c3 = c_in[3];
  uint32_t k0 = k_in[0], k1 = k_in[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* u = ((w >> 9) + 1/2) 2^-23: 2^23 equally spaced values strictly inside
 * (0,1), each exactly representable in single and double precision. */
double uniform_of(uint32_t w) { return ((double)(w >> 9) + 0.5) * (1.0 / 8388608.0); }

struct Stream {
  uint32_t key[2];
  uint32_t id_lo, id_hi;
  uint32_t block = 0;
  uint32_t words[4];
  int pos = 4;
  int drawn = 0;
  Stream(uint64_t seed, uint64_t id) {
    key[0] = (uint32_t)seed; key[1] = (uint32_t)(seed >> 32);
    id_lo = (uint32_t)id; id_hi = (uint32_t)(id >> 32);
  }
  double next() {
    if (pos == 4) {
      uint32_t ctr[4] = {block, id_lo, id_hi, 0u};
      philox(ctr, key, words);
      ++block;
      pos = 0;
    }
    ++drawn;
    return uniform_of(words[pos++]);
  }
};

/* -------------------------------------------------------------- nuclear masses
 * Sec. 2.2: binding energies from the semi-empirical mass formula (reading:
 * textbook coefficient set; measured values for A <= 4). */
double binding(int A, int Z) {
  if (A <= 0 || Z < 0 || Z > A) return 0.0;
  if (A <= 4) {
    if (A == 2 && Z == 1) return 2.224566;
    if (A == 3 && Z == 1) return 8.481798;
    if (A == 3 && Z == 2) return 7.718043;
    if (A == 4 && Z == 2) return 28.29566;
    return 0.0;
  }
  const int N = A - Z;
  const double a = (double)A;
  const double a13 = std::cbrt(a);
  double B = 15.75 * a - 17.8 * a13 * a13 - 0.711 * Z * (Z - 1) / a13 -
             23.7 * (double)(N - Z) * (N - Z) / a;
  if (Z % 2 == 0 && N % 2 == 0) B += 11.18 / std::sqrt(a);
  if (Z % 2 == 1 && N % 2 == 1) B -= 11.18 / std::sqrt(a);
  return B > 0.0 ? B : 0.0;
}

double mass(int A, int Z) { return Z * kMassP + (A - Z) * kMassN - binding(A, Z); }

/* ------------------------------------------------------------ nucleus setup
 * Sec. 2.2, Eq. (1): Fermi density with c = 1.07 A^1/3, delta = 0.545, outer
 * radius c + 2.5 fm, 15 equal shells whose densities come from integrating
 * rho(r) (reading: shell average, normalised so the shells hold A nucleons);
 * two-component Fermi gas (reading: local p_F per shell and species,
 * relativistic E_F); E_B = B/A; E_C = e^2 Z / R. */
double fermi_profile(double r, double c, double delta) { return 1.0 / (1.0 + std::exp((r - c) / delta)); }

double shell_integral(double r0, double r1, double c, double delta) {
  /* composite Simpson rule, 2000 intervals */
  const int n = 2000;
  const double h = (r1 - r0) / n;
  double s = 0.0;
  for (int k = 0; k <= n; ++k) {
    const double r = r0 + k * h;
    const double f = r * r * fermi_profile(r, c, delta);
    const double w = (k == 0 || k == n) ? 1.0 : ((k % 2) ? 4.0 : 2.0);
    s += w * f;
  }
  return s * h / 3.0;
}

void setup_nucleus(int A, int Z, const orc_options& opt, orc_nucleus& nu) {
  std::memset(&nu, 0, sizeof(nu));
  nu.A = A;
  nu.Z = Z;
  nu.c = 1.07 * std::cbrt((double)A);
  nu.delta = 0.545;
  nu.R = nu.c + 2.5;
  for (int i = 0; i <= ORC_NSHELL; ++i) nu.r[i] = nu.R * i / ORC_NSHELL;
  double total = 0.0;
  for (int i = 0; i < ORC_NSHELL; ++i) {
    nu.integral[i] = shell_integral(nu.r[i], nu.r[i + 1], nu.c, nu.delta);
    total += nu.integral[i];
  }
  const int N = A - Z;
  for (int i = 0; i < ORC_NSHELL; ++i) {
    const double vol = 4.0 / 3.0 * kPi * (std::pow(nu.r[i + 1], 3) - std::pow(nu.r[i], 3));
    double rho = A * (nu.integral[i] / total) / vol;
    if (opt.uniform_density) rho = A / (4.0 / 3.0 * kPi * std::pow(nu.R, 3));
    nu.rho[0][i] = rho * N / A;
    nu.rho[1][i] = rho * Z / A;
    for (int sp = 0; sp < 2; ++sp) {
      const double m = nucleon_mass(sp);
      double pF = kHbarC * std::cbrt(3.0 * kPi * kPi * nu.rho[sp][i]);
      if (opt.zero_fermi) pF = 0.0;
      nu.pF[sp][i] = pF;
      nu.EF[sp][i] = std::sqrt(pF * pF + m * m) - m;
    }
  }
  nu.EB = binding(A, Z) / A;
  nu.EC = kE2 * Z / nu.R;
  if (opt.zero_binding) {
    nu.EB = 0.0;
    nu.EC = 0.0;
  }
}

/* --------------------------------------------------------- NN cross-sections
 * Sec. 2.3: free elastic NN cross-sections of Cugnon et al.  Reading: the
 * recalled total cross-sections (p = p_lab in GeV/c, sigma in mb), with
 * max(low, middle branch) below 0.8 GeV/c, argument clamped to
 * [0.1374, 1.5] GeV/c; nn = pp, pn = np. */
double sig_like_low(double p) { return 34.0 * std::pow(p / 0.4, -2.104); }
double sig_like_mid(double p) { return 23.5 + 1000.0 * std::pow(p - 0.7, 4); }
double sig_like_high(double p) { return 1250.0 / (p + 50.0) - 4.0 * (p - 1.3) * (p - 1.3); }
double sig_unlike_low(double p) {
  const double l = std::log(p);
  return 6.3555 * std::pow(p, -3.2481) * std::exp(-0.377 * l * l);
}
double sig_unlike_mid(double p) { return 33.0 + 196.0 * std::pow(std::fabs(p - 0.95), 2.5); }
double sig_unlike_high(double p) { return 31.0 / std::sqrt(p); }

double clamp_p(double p) { return std::min(std::max(p, kPlo), kPhi); }

double sigma(int like, double p_in) {
  const double p = clamp_p(p_in);
  if (like) return p < 0.8 ? std::max(sig_like_low(p), sig_like_mid(p)) : sig_like_high(p);
  return p < 0.8 ? std::max(sig_unlike_low(p), sig_unlike_mid(p)) : sig_unlike_high(p);
}

/* Vertex of the concave like-pair branch above 0.8 GeV/c: root of
 * d/dp = -1250/(p+50)^2 - 8 (p - 1.3), by bisection. */
double like_high_vertex() {
  double lo = 0.8, hi = kPhi;
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    const double der = -1250.0 / ((mid + 50.0) * (mid + 50.0)) - 8.0 * (mid - 1.3);
    if (der > 0) lo = mid; else hi = mid;
  }
  return 0.5 * (lo + hi);
}

/* Majorant for the null-collision flight (reading): the maximum of sigma over
 * [pmin, 1.5 GeV/c].  Below 0.8 GeV/c both forms are convex (maximum at an
 * end point); above, the like-pair branch is concave (maximum at its vertex,
 * found by bisection) and the unlike one convex. */
double sigma_hat(int like, double pmin_in) {
  const double q = clamp_p(pmin_in);
  double m = sigma(like, q);
  if (q < 0.8) {
    const double left_of_08 = like ? std::max(sig_like_low(0.8), sig_like_mid(0.8))
                                   : std::max(sig_unlike_low(0.8), sig_unlike_mid(0.8));
    m = std::max(m, left_of_08);
  }
  const double a = std::max(q, 0.8);
  if (like) {
    static const double vertex = like_high_vertex();
    m = std::max(m, sig_like_high(std::min(std::max(vertex, a), kPhi)));
  } else {
    m = std::max(m, sig_unlike_high(a));
  }
  return m;
}

/* Sec. 2.3: differential elastic cross-section d sigma/dt ~ exp(b t)
 * (reading: recalled Cugnon slopes, (GeV/c)^-2). */
double slope(int like, double p_in) {
  const double p = clamp_p(p_in);
  if (like) {
    const double p8 = std::pow(p, 8);
    return 5.5 * p8 / (7.7 + p8);
  }
  if (p < 0.225) return 0.0;
  if (p < 0.6) return 16.53 * (p - 0.225);
  return -1.63 * p + 7.16;
}

/* Smallest momentum of x in the rest frame of a target y taken from a Fermi
 * sphere of radius pF: collinear target at the largest reachable rapidity. */
double plab_min(double p, double mx, double pF, double my) {
  const double Ex = std::sqrt(p * p + mx * mx);
  const double EFy = std::sqrt(pF * pF + my * my);
  const double v = (p * EFy - Ex * pF) / my;
  return v > 0.0 ? v : 0.0;
}

/* --------------------------------------------------------------- kinematics */
struct Vec3 { double x, y, z; };
inline Vec3 operator+(Vec3 a, Vec3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
inline Vec3 operator-(Vec3 a, Vec3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline Vec3 operator*(double s, Vec3 a) { return {s * a.x, s * a.y, s * a.z}; }
inline double dot(Vec3 a, Vec3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline double norm(Vec3 a) { return std::sqrt(dot(a, a)); }
inline Vec3 cross(Vec3 a, Vec3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }

inline double kinetic(double p, double m) { return p * p / (std::sqrt(p * p + m * m) + m); }

/* Sec. 2.2: target momentum from the "quadratic distribution", P(p) ~ p^2 on
 * [0, p_F] (reading: uniform in the local Fermi sphere, isotropic).  Uniforms
 * in stream order: u_mag (|p| = p_F u^1/3), u_cos (cos theta = 2u - 1),
 * u_phi (phi = 2 pi u).  *mag receives |p|. */
Vec3 fermi_sample(double pF, double u_mag, double u_cos, double u_phi, double* mag) {
  const double pt_mag = pF * std::cbrt(u_mag);
  const double ct = 2.0 * u_cos - 1.0;
  const double st = std::sqrt(std::max(0.0, 1.0 - ct * ct));
  const double ph = 2.0 * kPi * u_phi;
  *mag = pt_mag;
  return pt_mag * Vec3{st * std::cos(ph), st * std::sin(ph), ct};
}

/* Unit vector at polar angle theta (cos c, sin s) and azimuth phi from a. */
Vec3 rotate(Vec3 a, double c, double s, double phi) {
  const double st = std::sqrt(a.x * a.x + a.y * a.y);
  const double cp = std::cos(phi), sp = std::sin(phi);
  if (st > 1e-6) {
    Vec3 e1 = {a.x * a.z / st, a.y * a.z / st, -st};
    Vec3 e2 = {-a.y / st, a.x / st, 0.0};
    return c * a + s * (cp * e1 + sp * e2);
  }
  return {s * cp, s * sp, a.z >= 0 ? c : -c};
}

/* Lorentz boost of a momentum q (mass m) from a frame moving with
 * gamma*beta = u (gamma = g) back to the lab. */
void boost(Vec3 q, double m, Vec3 u, double g, Vec3& p_lab, double& T_lab) {
  const double E = std::sqrt(dot(q, q) + m * m);
  const double uq = dot(u, q);
  p_lab = q + (uq / (g + 1.0) + E) * u;
  const double Tstar = kinetic(norm(q), m);
  T_lab = g * Tstar + dot(u, u) / (g + 1.0) * m + uq;
}

/* Sec. 2.3: fully relativistic two-body elastic scattering.  CM polar angle
 * from d sigma/dt ~ exp(b t), t = -2 p*^2 (1 - cos theta*) (reading). */
double elastic(Vec3 px, double mx, Vec3 pt, double my, double b, double u_theta, double u_phi,
               Vec3& qx, Vec3& qt, double& Tx_out, double& Tt_out) {
  const double Tx = kinetic(norm(px), mx), Tt = kinetic(norm(pt), my);
  const Vec3 P = px + pt;
  const double Q = 2.0 * (Tx * Tt + Tx * my + Tt * mx - dot(px, pt));
  const double s = (mx + my) * (mx + my) + Q;
  const double rs = std::sqrt(s);
  const double pstar = std::sqrt(Q * (Q + 4.0 * mx * my) / (4.0 * s));
  const double plab = pstar * rs / my;
  const Vec3 u = (1.0 / rs) * P;
  const double g = (Tx + Tt + mx + my) / rs;
  /* direction of x in the CM frame */
  const Vec3 qcm = px + (dot(u, px) / (g + 1.0) - (Tx + mx)) * u;
  const Vec3 a = (1.0 / norm(qcm)) * qcm;
  const double k = 2.0 * b * (pstar / 1000.0) * (pstar / 1000.0);
  double y = (k < 1e-6) ? 2.0 * u_theta : -std::log1p(u_theta * std::expm1(-2.0 * k)) / k;
  y = std::min(std::max(y, 0.0), 2.0);
  const double c = 1.0 - y;
  const double sn = std::sqrt(std::max(0.0, y * (2.0 - y)));
  const Vec3 n = rotate(a, c, sn, 2.0 * kPi * u_phi);
  boost(pstar * n, mx, u, g, qx, Tx_out);
  boost((-pstar) * n, my, u, g, qt, Tt_out);
  return plab;
}

/* Reading of the Chen et al. prescription (Sec. 2.3): at a potential step the
 * tangential momentum is kept and T - V is conserved; the particle is
 * reflected when the normal component cannot be formed. */
int refract(Vec3& d, Vec3 n, double T_from, double T_to, double m) {
  const double p_from = std::sqrt(T_from * T_from + 2.0 * T_from * m);
  const double pn = p_from * dot(d, n);
  if (T_to > 0.0) {
    const double dp2 = (T_to - T_from) * (T_to + T_from + 2.0 * m);
    const double pn2 = pn * pn + dp2;
    if (pn2 > 0.0) {
      const Vec3 p = p_from * d;
      const Vec3 pt = p - pn * n;
      const double pn_new = (pn >= 0 ? 1.0 : -1.0) * std::sqrt(pn2);
      const Vec3 q = pt + pn_new * n;
      d = (1.0 / norm(q)) * q;
      return 1;
    }
  }
  d = d - (2.0 * dot(d, n)) * n;
  return 0;
}

/* ----------------------------------------------------------- evaporation
 * Sec. 2.4 with Weisskopf-Ewing widths (reading): Gamma_j ~ g_j m_j R_j^2
 * I(a, U_j), I(a,U) = int_0^U x exp(2 sqrt(a (U-x))) dx. */
double width_integral(double a, double U) {
  if (U <= 0.0) return 0.0;
  const double Y = 2.0 * std::sqrt(a * U);
  if (Y < 2.0) {
    /* (1/4a^2) sum_{n>=4} (n-1)(n-3) Y^n / n! */
    double term = std::pow(Y, 4) / 24.0;  /* Y^n/n! at n = 4 */
    double sum = 0.0;
    for (int n = 4; n < 60; ++n) {
      sum += (n - 1) * (n - 3) * term;
      term *= Y / (n + 1);
    }
    return sum / (4.0 * a * a);
  }
  return (std::exp(Y) * (2.0 * Y * Y - 6.0 * Y + 6.0) + Y * Y - 6.0) / (8.0 * a * a);
}

/* J(y) = int_0^y (Y^2 - s^2) s e^s ds; closed form G(y) - G(0) with
 * G(y) = e^y [Y^2 (y - 1) - (y^3 - 3 y^2 + 6 y - 6)], series for small Y. */
double spectrum_J(double y, double Y) {
  if (Y < 2.0) {
    double sum = 0.0, fact = 1.0, yn = 1.0;
    for (int n = 0; n < 60; ++n) {
      sum += (Y * Y * yn * y * y / (n + 2) - yn * y * y * y * y / (n + 4)) / fact;
      fact *= (n + 1);
      yn *= y;
    }
    return sum;
  }
  const double G = std::exp(y) * (Y * Y * (y - 1.0) - (y * y * y - 3.0 * y * y + 6.0 * y - 6.0));
  const double G0 = -Y * Y + 6.0;
  return G - G0;
}

/* CDF of the kinetic-energy excess x in [0,U]: density ~ x rho(U - x). */
double spectrum_cdf(double a, double U, double x) {
  if (x <= 0.0) return 0.0;
  if (x >= U) return 1.0;
  const double Y = 2.0 * std::sqrt(a * U);
  const double y = 2.0 * std::sqrt(a * (U - x));
  const double JY = spectrum_J(Y, Y);
  return (JY - spectrum_J(y, Y)) / JY;
}

double spectrum_sample(double a, double U, double u) {
  double lo = 0.0, hi = U;
  for (int it = 0; it < 200 && hi - lo > 1e-15 * U; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (spectrum_cdf(a, U, mid) < u) lo = mid; else hi = mid;
  }
  return 0.5 * (lo + hi);
}

struct Fragment { int a, z, g; };
constexpr Fragment kFrag[6] = {{1, 0, 2}, {1, 1, 2}, {2, 1, 3}, {3, 1, 2}, {3, 2, 2}, {4, 2, 1}};

/* Reading R20 (option heavy_fragments): GEM's ejectiles reach Mg (Sec. 2.4);
 * the heavier ones emitted here are the stable isotopes of Li to Mg with
 * their measured ground-state spins (g = 2s + 1), as channels 7-26, with the
 * particles' width and spectrum (R15) and masses from the same mass formula. */
constexpr Fragment kHeavy[20] = {{6, 3, 3},   {7, 3, 4},   {9, 4, 4},   {10, 5, 7},  {11, 5, 4},
                                 {12, 6, 1},  {13, 6, 2},  {14, 7, 3},  {15, 7, 2},  {16, 8, 1},
                                 {17, 8, 6},  {18, 8, 1},  {19, 9, 2},  {20, 10, 1}, {21, 10, 4},
                                 {22, 10, 1}, {23, 11, 4}, {24, 12, 1}, {25, 12, 6}, {26, 12, 1}};
constexpr int kNumChan = 27;  /* 0-5 particles, 6 photon, 7-26 heavier fragments */

/* Fragment of channel j; false for the photon (6) and out of range. */
bool fragment_of(int j, Fragment& f) {
  if (j >= 0 && j < 6) {
    f = kFrag[j];
    return true;
  }
  if (j >= 7 && j < kNumChan) {
    f = kHeavy[j - 7];
    return true;
  }
  return false;
}

/* ------------------------------------------------ photon emission (option)
 * Reading R19.  Sec. 2 has an excited nucleus shed its energy by particle
 * emission first, then by photons; Sec. 2.4 leaves photon evaporation out,
 * so it is an option, off by default.  The photon channel competes with the
 * six particle channels at every step.  Detailed balance with two photon
 * polarisations gives, in the units of the particle widths above (which are
 * Gamma_j pi (hbar c)^2 rho(E)),
 *   w_gamma = (1/pi) int_0^E eps^2 sigma_g(eps) rho(E - eps) d eps,
 * with the same level density rho(U) = exp(2 sqrt(a U)), a = A/8 of the
 * nucleus itself (a photon leaves A and Z unchanged).  The photoabsorption
 * cross-section rises linearly, sigma_g = s0 eps, up to the giant-dipole
 * energy E_G = 31.2 A^-1/3 + 20.6 A^-1/6 MeV so that the ramp holds the
 * classical dipole sum 60 N Z / A mb MeV: s0 = 12 N Z / (A E_G^2) fm^2/MeV
 * (1 mb = 0.1 fm^2).  Then w_gamma = (s0/pi) J(a, E), J(a, U) =
 * int_0^U eps^3 exp(2 sqrt(a (U - eps))) d eps.  The channel is open while
 * E > 0.1 MeV; below that the rest of E stays with the nucleus.  A nucleus
 * with N = 0 or Z = 0 has no dipole strength (s0 = 0): no photons. */
constexpr double kPhotonMin = 0.1;

double gdr_energy(int A) { return 31.2 / std::cbrt((double)A) + 20.6 / std::pow((double)A, 1.0 / 6.0); }

double photon_s0(int A, int Z) {
  const double EG = gdr_energy(A);
  return 12.0 * (double)(A - Z) * (double)Z / ((double)A * EG * EG);
}

/* L(y, Y) = int_0^y (Y^2 - t^2)^3 t e^t dt.  The polynomial is
 * Y^6 t - 3 Y^4 t^3 + 3 Y^2 t^5 - t^7.  Small Y: the series of e^t, term
 * by term; otherwise the antiderivative e^t sum_j (-1)^j P^(j)(t). */
double photon_L(double y, double Y) {
  double c[8] = {0.0, std::pow(Y, 6), 0.0, -3.0 * std::pow(Y, 4), 0.0, 3.0 * Y * Y, 0.0, -1.0};
  if (Y < 10.0) {
    double sum = 0.0, fact = 1.0;
    for (int n = 0; n < 90; ++n) {
      double inner = 0.0;  /* int_0^y P(t) t^n dt */
      for (int k = 1; k < 8; k += 2) inner += c[k] * std::pow(y, k + n + 1) / (k + n + 1);
      sum += inner / fact;
      fact *= (n + 1);
    }
    return sum;
  }
  auto G = [&](double t) {
    /* e^t sum_j (-1)^j P^(j)(t), derivatives of the coefficient array */
    double d[8];
    std::memcpy(d, c, sizeof(d));
    double acc = 0.0, sign = 1.0;
    for (int j = 0; j < 8; ++j) {
      double v = 0.0;
      for (int k = 7; k >= 0; --k) v = v * t + d[k];
      acc += sign * v;
      sign = -sign;
      for (int k = 0; k < 7; ++k) d[k] = (k + 1) * d[k + 1];
      d[7] = 0.0;
    }
    return std::exp(t) * acc;
  };
  return G(y) - G(0.0);
}

/* J(a, U) = int_0^U eps^3 exp(2 sqrt(a (U - eps))) d eps: with
 * y = 2 sqrt(a (U - eps)), J = L(Y, Y) / (128 a^4), Y = 2 sqrt(a U); a -> 0
 * gives U^4 / 4. */
double photon_J(double a, double U) {
  if (U <= 0.0) return 0.0;
  if (a <= 0.0) return U * U * U * U / 4.0;
  const double Y = 2.0 * std::sqrt(a * U);
  return photon_L(Y, Y) / (128.0 * a * a * a * a);
}

/* CDF of the photon's energy share eps in [0, U]: density ~ eps^3 rho(U - eps). */
double photon_cdf(double a, double U, double x) {
  if (x <= 0.0) return 0.0;
  if (x >= U) return 1.0;
  if (a <= 0.0) return std::pow(x / U, 4);
  const double Y = 2.0 * std::sqrt(a * U);
  const double y = 2.0 * std::sqrt(a * (U - x));
  const double LY = photon_L(Y, Y);
  return (LY - photon_L(y, Y)) / LY;
}

double photon_sample(double a, double U, double u) {
  double lo = 0.0, hi = U;
  for (int it = 0; it < 200 && hi - lo > 1e-15 * U; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (photon_cdf(a, U, mid) < u) lo = mid; else hi = mid;
  }
  return 0.5 * (lo + hi);
}

/* photon channel weight of nucleus (A, Z) at excitation E (0: closed) */
double photon_width(int A, int Z, double E) {
  if (!(E > kPhotonMin)) return 0.0;
  return photon_s0(A, Z) / kPi * photon_J(A / 8.0, E);
}

/* Sec. 2.3 after an elastic NN collision in shell s between a moving nucleon
 * of species sx and a target of species sy (0 n, 1 p), with product kinetic
 * energies Tx (the moving nucleon's) and Ty (the struck one's) and the
 * target's kinetic energy Tt before the collision.
 * Pauli: the collision happens only when both products end above the Fermi
 * energy of their own species in that shell (reading: strict, local).
 * Then each product's excess energy eps = T - E_F(own species, s) decides the
 * cutoff: it stays in the nucleus (captured) when eps < E_B, plus E_C for a
 * proton; otherwise it is tracked.  The hole left in the target's Fermi sea
 * is E_F(sy, s) - Tt (reading: energy bookkeeping of the excitation). */
struct CollisionOutcome {
  bool blocked;
  bool track_x, track_y;
  double eps_x, eps_y, hole;
};

double cutoff_energy(const orc_nucleus& nu, int sp) { return nu.EB + (sp == 1 ? nu.EC : 0.0); }

CollisionOutcome collision_outcome(const orc_nucleus& nu, int s, int sx, int sy, double Tx, double Ty, double Tt,
                                   bool pauli) {
  CollisionOutcome o;
  o.blocked = pauli && (Tx <= nu.EF[sx][s] || Ty <= nu.EF[sy][s]);
  o.hole = std::max(0.0, nu.EF[sy][s] - Tt);
  o.eps_x = Tx - nu.EF[sx][s];
  o.eps_y = Ty - nu.EF[sy][s];
  o.track_x = o.eps_x >= cutoff_energy(nu, sx);
  o.track_y = o.eps_y >= cutoff_energy(nu, sy);
  return o;
}

/* ------------------------------------------------------------------- events */
struct Particle {
  Vec3 pos, d;
  double eps;   /* T - E_F (local): invariant under refraction (reading) */
  int sp;       /* 0 n, 1 p */
  int shell;    /* 0 .. 14 */
};

struct Event {
  const orc_nucleus& nu;
  const orc_options& opt;
  Stream rng;
  orc_result& res;
  std::vector<orc_secondary>& out;
  uint32_t event_index;
  int max_stack, max_seg;

  double Ex = 0.0;
  Vec3 pres = {0, 0, 0};
  int n_esc[2] = {0, 0};
  /* nucleons of each species still in the Fermi sea: a struck nucleon
   * leaves it, a captured particle returns to it (reading) */
  int avail[2];
  int sea_min = 0;
  double sh[2] = {0, 0};  /* majorant cross-sections (fm^2) for targets n, p */

  Event(const orc_nucleus& n_, const orc_options& o, uint64_t seed, uint64_t id, orc_result& r,
        std::vector<orc_secondary>& v, uint32_t idx)
      : nu(n_), opt(o), rng(seed, id), res(r), out(v), event_index(idx) {
    max_stack = opt.max_stack > 0 ? opt.max_stack : 64;
    max_seg = opt.max_segments > 0 ? opt.max_segments : 10000;
  }

  /* majorant for a flight of species x with excess energy eps (reading) */
  void set_majorant(const Particle& q) {
    res.n_majorant++;
    const double mx = nucleon_mass(q.sp);
    double EFmin = nu.EF[q.sp][0];
    for (int i = 1; i < ORC_NSHELL; ++i) EFmin = std::min(EFmin, nu.EF[q.sp][i]);
    const double T = q.eps + EFmin;
    const double p = std::sqrt(T * T + 2.0 * T * mx);
    for (int y = 0; y < 2; ++y) {
      double pFmax = nu.pF[y][0];
      for (int i = 1; i < ORC_NSHELL; ++i) pFmax = std::max(pFmax, nu.pF[y][i]);
      const double pmin = plab_min(p, mx, pFmax, nucleon_mass(y)) / 1000.0;
      const double s_mb = opt.const_sigma_mb > 0 ? opt.const_sigma_mb : sigma_hat(q.sp == y, pmin);
      sh[y] = s_mb * kMbToFm2;
    }
  }

  /* optical depth of a new flight segment sequence (reading): -ln u */
  double new_tau() {
    res.n_tau++;
    return -std::log(rng.next());
  }

  double weight(int y, int shell) const {
    if (avail[y] <= 0) return 0.0;   /* no nucleon of species y left in the sea */
    return nu.rho[y][shell] * sh[y];
  }

  /* cutoff (Sec. 2.3): the particle stays in the nucleus, its excess energy
   * goes to the excitation energy */
  void capture(const Particle& q) {
    Ex += q.eps;
    avail[q.sp]++;
  }

  /* a collision takes a nucleon of species y out of the sea; the lowest
   * occupancy reached is kept for the sea-occupancy check (reading) */
  void strike(int y) {
    avail[y]--;
    sea_min = std::min(sea_min, avail[y]);
  }

  void emit(int sp, int stage, double T, Vec3 d) {
    orc_secondary s;
    std::memset(&s, 0, sizeof(s));
    s.event = event_index;
    s.species = sp;
    s.stage = stage;
    s.T = T;
    s.u[0] = d.x; s.u[1] = d.y; s.u[2] = d.z;
    out.push_back(s);
    res.n_sec++;
  }

  /* One cascade attempt.  Returns true when at least one collision happened. */
  bool cascade_pass(double T0) {
    std::vector<Particle> stack;
    std::vector<orc_secondary> pass_out;
    /* entry (reading): b uniform over the disc, inward refraction at R */
    const double ub = rng.next(), uphi = rng.next();
    double b = nu.R * std::sqrt(ub);
    if (opt.fixed_b >= 0) b = opt.fixed_b;
    const double phi = 2.0 * kPi * uphi;
    Particle cur;
    cur.pos = {b * std::cos(phi), b * std::sin(phi), -std::sqrt(std::max(0.0, nu.R * nu.R - b * b))};
    cur.d = {0.0, 0.0, 1.0};
    cur.eps = T0 + nu.EB;
    cur.sp = 1;
    cur.shell = ORC_NSHELL - 1;
    {
      const double r = norm(cur.pos);
      const Vec3 n = r > 0 ? (1.0 / r) * cur.pos : Vec3{0, 0, -1};
      refract(cur.d, n, T0, cur.eps + nu.EF[1][ORC_NSHELL - 1], kMassP);
    }
    set_majorant(cur);
    double tau = new_tau();
    bool have = true;

    while (have) {
      if (res.n_seg >= max_seg) {
        /* segment guard: capture everything still moving */
        res.flags |= 2;
        capture(cur);
        for (const Particle& q : stack) capture(q);
        stack.clear();
        if (res.n_coll == 0) return true;  /* ends the event as a capture */
        break;
      }
      res.n_seg++;
      const int s = cur.shell;
      const double lam = weight(0, s) + weight(1, s);
      const double xd = dot(cur.pos, cur.d);
      const Vec3 cx = cross(cur.pos, cur.d);
      const double b2 = dot(cx, cx);
      double t;
      int dest;
      const double rin = nu.r[s], rout = nu.r[s + 1];
      if (s > 0 && xd < 0 && b2 < rin * rin) {
        t = std::max(0.0, -xd - std::sqrt(rin * rin - b2));
        dest = s - 1;
      } else {
        t = std::max(0.0, -xd + std::sqrt(std::max(0.0, rout * rout - b2)));
        dest = s + 1;
      }
      if (tau < lam * t) {
        /* tentative collision (null-collision flight, reading) */
        cur.pos = cur.pos + (tau / lam) * cur.d;
        res.n_tent++;
        res.tent_shells = res.tent_shells * 3u + (uint32_t)(s + 1);
        const double w0 = weight(0, s), w1 = weight(1, s);
        const int y = (w0 > rng.next() * (w0 + w1)) ? 0 : 1;
        const double mx = nucleon_mass(cur.sp), my = nucleon_mass(y);
        /* target momentum: uniform in the local Fermi sphere (Sec. 2.2) */
        const double u_mag = rng.next(), u_cos = rng.next(), u_phi = rng.next();
        double pt_mag;
        const Vec3 pt = fermi_sample(nu.pF[y][s], u_mag, u_cos, u_phi, &pt_mag);
        const double Tx = cur.eps + nu.EF[cur.sp][s];
        const Vec3 px = std::sqrt(Tx * Tx + 2.0 * Tx * mx) * cur.d;
        const int like = (cur.sp == y);
        /* p_lab of x in the rest frame of y */
        const double Tt = kinetic(pt_mag, my);
        const double Q = 2.0 * (Tx * Tt + Tx * my + Tt * mx - dot(px, pt));
        const double ss = (mx + my) * (mx + my) + Q;
        const double plab = std::sqrt(Q * (Q + 4.0 * mx * my) / (4.0 * ss)) * std::sqrt(ss) / my;
        const double sig = (opt.const_sigma_mb > 0 ? opt.const_sigma_mb : sigma(like, plab / 1000.0)) * kMbToFm2;
        const double u_acc = rng.next();
        if (!(u_acc < sig / sh[y])) {
          tau = new_tau();
          continue;
        }
        const double u_th = rng.next(), u_ph = rng.next();
        Vec3 qx, qt;
        double Txn, Ttn;
        elastic(px, mx, pt, my, slope(like, plab / 1000.0), u_th, u_ph, qx, qt, Txn, Ttn);
        if (like && rng.next() < 0.5) {
          std::swap(qx, qt);
          std::swap(Txn, Ttn);
        }
        const CollisionOutcome oc = collision_outcome(nu, s, cur.sp, y, Txn, Ttn, Tt, !opt.no_pauli);
        if (oc.blocked) {
          res.n_pauli++;
          tau = new_tau();
          continue;
        }
        /* accepted collision: the struck nucleon leaves the sea */
        res.n_coll++;
        strike(y);
        Ex += oc.hole;
        if (res.n_coll == 1) res.first_z = cur.pos.z;
        Particle px_new = cur, py_new = cur;
        px_new.d = (1.0 / norm(qx)) * qx;
        px_new.eps = oc.eps_x;
        py_new.d = (1.0 / norm(qt)) * qt;
        py_new.sp = y;
        py_new.eps = oc.eps_y;
        if (opt.stop_after_first) {
          capture(px_new);
          capture(py_new);
          for (const Particle& q : stack) capture(q);
          stack.clear();
          break;
        }
        const bool tx = oc.track_x;
        const bool ty = oc.track_y;
        if (!tx) capture(px_new);
        if (!ty) capture(py_new);
        if (tx && ty) {
          if ((int)stack.size() >= max_stack) {
            res.flags |= 1;
            capture(py_new);
          } else {
            stack.push_back(py_new);
          }
          cur = px_new;
        } else if (tx) {
          cur = px_new;
        } else if (ty) {
          cur = py_new;
        } else {
          if (stack.empty()) { have = false; break; }
          cur = stack.back();
          stack.pop_back();
        }
        set_majorant(cur);
        tau = new_tau();
        continue;
      }
      /* reach the boundary */
      tau -= lam * t;
      cur.pos = cur.pos + t * cur.d;
      const double r = norm(cur.pos);
      const Vec3 n = (1.0 / r) * cur.pos;
      const double m = nucleon_mass(cur.sp);
      const double T_from = cur.eps + nu.EF[cur.sp][s];
      if (dest == ORC_NSHELL) {
        const double T_out = cur.eps - nu.EB;
        if (refract(cur.d, n, T_from, T_out, m)) {
          if (res.n_coll == 0) return false;  /* transparent pass */
          const double p = std::sqrt(T_out * T_out + 2.0 * T_out * m);
          pres = pres - p * cur.d;
          n_esc[cur.sp]++;
          emit(cur.sp, 0, T_out, cur.d);
          if (stack.empty()) { have = false; break; }
          cur = stack.back();
          stack.pop_back();
          set_majorant(cur);
          tau = new_tau();
        }
      } else {
        if (refract(cur.d, n, T_from, cur.eps + nu.EF[cur.sp][dest], m)) cur.shell = dest;
      }
    }
    return true;
  }

  void evaporate(int A, int Z, double E, Vec3 P) {
    while (true) {
      /* channels 0-5: the particles of kFrag; 6: a photon (option, R19);
       * 7-26: the heavier fragments of kHeavy (option, R20) */
      double w[kNumChan], U[kNumChan], V[kNumChan], a[kNumChan];
      int Ad[kNumChan], Zd[kNumChan];
      double total = 0.0;
      for (int j = 0; j < kNumChan; ++j) {
        w[j] = 0.0;
        Fragment f;
        if (!fragment_of(j, f) || (j >= 7 && !opt.heavy_fragments)) continue;
        Ad[j] = A - f.a;
        Zd[j] = Z - f.z;
        if (Ad[j] < 1 || Zd[j] < 0 || Zd[j] > Ad[j]) continue;
        const double S = binding(A, Z) - binding(Ad[j], Zd[j]) - binding(f.a, f.z);
        const double ad13 = std::cbrt((double)Ad[j]);
        const double aj13 = std::cbrt((double)f.a);
        V[j] = f.z > 0 ? kE2 * f.z * Zd[j] / (1.5 * (ad13 + aj13)) : 0.0;
        U[j] = E - S - V[j];
        if (!(U[j] > 0.0)) continue;
        a[j] = Ad[j] / 8.0;
        const double Rj = j <= 1 ? 1.5 * ad13 : 1.5 * (ad13 + aj13);
        w[j] = f.g * mass(f.a, f.z) * Rj * Rj * width_integral(a[j], U[j]);
        total += w[j];
      }
      w[6] = opt.photon_evaporation ? photon_width(A, Z, E) : 0.0;
      total += w[6];
      if (!(total > 0.0)) break;
      const double uc = rng.next() * total;
      int j = 0;
      double cum = 0.0;
      for (j = 0; j < kNumChan; ++j) {
        cum += w[j];
        if (w[j] > 0.0 && cum > uc) break;
      }
      if (j == kNumChan) {  /* rounding at the top: take the last open channel */
        for (j = kNumChan - 1; j >= 0 && !(w[j] > 0.0); --j) {}
      }
      if (j == 6) {
        /* photon: eps from its spectrum, A and Z unchanged; in the nucleus's
         * rest frame the photon carries (Mp^2 - Md^2) / (2 Mp) */
        const double x = photon_sample(A / 8.0, E, rng.next());
        const double Ed = E - x;
        const double Mp = mass(A, Z) + E;
        const double Md = mass(A, Z) + Ed;
        const double Eg = x * (Mp + Md) / (2.0 * Mp);
        const double ct = 2.0 * rng.next() - 1.0;
        const double st = std::sqrt(std::max(0.0, 1.0 - ct * ct));
        const double ph = 2.0 * kPi * rng.next();
        const Vec3 q = Eg * Vec3{st * std::cos(ph), st * std::sin(ph), ct};
        const Vec3 u = (1.0 / Mp) * P;
        const double g = std::sqrt(1.0 + dot(u, u));
        Vec3 pf;
        double Tf;
        boost(q, 0.0, u, g, pf, Tf);
        res.n_evap++;
        emit(6, 1, Tf, (1.0 / norm(pf)) * pf);
        P = P - pf;
        E = Ed;
        continue;
      }
      Fragment f;
      fragment_of(j, f);
      const double x = spectrum_sample(a[j], U[j], rng.next());
      const double Ed = U[j] - x;
      const double eps = V[j] + x;
      const double Mp = mass(A, Z) + E;
      const double Mb = mass(Ad[j], Zd[j]) + Ed;
      const double mc = mass(f.a, f.z);
      const double p2 = eps * (eps + 2.0 * mc) * (eps + 2.0 * Mb) * (eps + 2.0 * Mb + 2.0 * mc) / (4.0 * Mp * Mp);
      const double ps = std::sqrt(p2);
      const double ct = 2.0 * rng.next() - 1.0;
      const double st = std::sqrt(std::max(0.0, 1.0 - ct * ct));
      const double ph = 2.0 * kPi * rng.next();
      const Vec3 q = ps * Vec3{st * std::cos(ph), st * std::sin(ph), ct};
      const Vec3 u = (1.0 / Mp) * P;
      const double g = std::sqrt(1.0 + dot(u, u));
      Vec3 pf;
      double Tf;
      boost(q, mc, u, g, pf, Tf);
      res.n_evap++;
      emit(j, 1, Tf, (1.0 / norm(pf)) * pf);
      P = P - pf;
      A = Ad[j];
      Z = Zd[j];
      E = Ed;
    }
    res.A_f = A;
    res.Z_f = Z;
    res.Ex_f = E;
    res.p_f[0] = P.x; res.p_f[1] = P.y; res.p_f[2] = P.z;
  }

  void run(double T0) {
    std::memset(&res, 0, sizeof(res));
    res.first_z = NAN;
    const size_t mark = out.size();
    while (true) {
      Ex = 0.0;
      pres = {0, 0, 0};
      n_esc[0] = n_esc[1] = 0;
      avail[0] = nu.A - nu.Z;   /* the projectile proton is out of the sea */
      avail[1] = nu.Z;
      sea_min = std::min(avail[0], avail[1]);
      out.resize(mark);
      res.n_sec = 0;
      if (cascade_pass(T0)) break;
      res.n_retry++;
    }
    const double p0 = std::sqrt(T0 * T0 + 2.0 * T0 * kMassP);
    pres = pres + Vec3{0, 0, p0};
    res.A_casc = nu.A + 1 - n_esc[0] - n_esc[1];
    res.Z_casc = nu.Z + 1 - n_esc[1];
    res.Ex_casc = Ex;
    res.p_casc[0] = pres.x; res.p_casc[1] = pres.y; res.p_casc[2] = pres.z;
    res.sea[0] = avail[0];
    res.sea[1] = avail[1];
    res.sea_min = sea_min;
    if (res.A_casc <= 0) {
      res.flags |= 4;
      res.A_f = res.A_casc; res.Z_f = res.Z_casc; res.Ex_f = Ex;
      std::memcpy(res.p_f, res.p_casc, sizeof(res.p_f));
    } else if (opt.no_evaporation) {
      res.A_f = res.A_casc; res.Z_f = res.Z_casc; res.Ex_f = Ex;
      std::memcpy(res.p_f, res.p_casc, sizeof(res.p_f));
    } else {
      evaporate(res.A_casc, res.Z_casc, Ex, pres);
    }
    res.n_draw = rng.drawn;
  }
};

}  // namespace

/* ==================================================================== C ABI */
extern "C" {

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) { philox(ctr, key, out); }
double orc_uniform(uint32_t w) { return uniform_of(w); }
double orc_stream_uniform(uint64_t seed, uint64_t event_id, uint64_t k) {
  /* the k-th draw of the stream the events use */
  Stream st(seed, event_id);
  for (uint64_t i = 0; i < k; ++i) st.next();
  return st.next();
}
double orc_binding(int A, int Z) { return binding(A, Z); }
double orc_mass(int A, int Z) { return mass(A, Z); }
int orc_nucleus_setup(int A, int Z, const orc_options* opt, orc_nucleus* out) {
  if (A < 4 || A > 250 || Z < 1 || Z >= A || !out) return -1;
  orc_options zero;
  std::memset(&zero, 0, sizeof(zero));
  zero.fixed_b = -1.0;
  setup_nucleus(A, Z, opt ? *opt : zero, *out);
  return 0;
}
double orc_sigma(int like, double p) { return sigma(like, p); }
double orc_sigma_hat(int like, double p) { return sigma_hat(like, p); }
double orc_slope(int like, double p) { return slope(like, p); }
double orc_plab_min(double p, double mx, double pF, double my) { return plab_min(p, mx, pF, my); }

double orc_elastic(const double px[3], double mx, const double pt[3], double my, double b,
                   double u_theta, double u_phi, double qx[3], double qt[3], double* Tx, double* Tt) {
  Vec3 a, c;
  const double plab = elastic({px[0], px[1], px[2]}, mx, {pt[0], pt[1], pt[2]}, my, b, u_theta, u_phi, a, c, *Tx, *Tt);
  qx[0] = a.x; qx[1] = a.y; qx[2] = a.z;
  qt[0] = c.x; qt[1] = c.y; qt[2] = c.z;
  return plab;
}

int orc_refract(double d[3], const double n[3], double T_from, double T_to, double m) {
  Vec3 v = {d[0], d[1], d[2]};
  const int r = refract(v, {n[0], n[1], n[2]}, T_from, T_to, m);
  d[0] = v.x; d[1] = v.y; d[2] = v.z;
  return r;
}

int orc_collision_outcome(const orc_nucleus* nu, int shell, int sp_x, int sp_y, double Tx, double Ty, double Tt,
                          int pauli, double out[3]) {
  if (!nu || !out || shell < 0 || shell >= ORC_NSHELL || sp_x < 0 || sp_x > 1 || sp_y < 0 || sp_y > 1) return -1;
  const CollisionOutcome o = collision_outcome(*nu, shell, sp_x, sp_y, Tx, Ty, Tt, pauli != 0);
  out[0] = o.eps_x;
  out[1] = o.eps_y;
  out[2] = o.hole;
  return (o.blocked ? 1 : 0) | (o.track_x ? 2 : 0) | (o.track_y ? 4 : 0);
}

double orc_width_integral(double a, double U) { return width_integral(a, U); }
double orc_spectrum_cdf(double a, double U, double x) { return spectrum_cdf(a, U, x); }
double orc_spectrum_sample(double a, double U, double u) { return spectrum_sample(a, U, u); }
double orc_gdr_energy(int A) { return gdr_energy(A); }
double orc_photon_s0(int A, int Z) { return photon_s0(A, Z); }
double orc_photon_integral(double a, double U) { return photon_J(a, U); }
double orc_photon_cdf(double a, double U, double x) { return photon_cdf(a, U, x); }
double orc_photon_sample(double a, double U, double u) { return photon_sample(a, U, u); }
double orc_photon_width(int A, int Z, double E) { return photon_width(A, Z, E); }
int orc_fragment(int j, int* a, int* z, int* g) {
  Fragment f;
  if (!fragment_of(j, f)) return 0;
  if (a) *a = f.a;
  if (z) *z = f.z;
  if (g) *g = f.g;
  return 1;
}

void orc_fermi_sample(double pF, double u1, double u2, double u3, double p[3]) {
  double mag;
  const Vec3 v = fermi_sample(pF, u1, u2, u3, &mag);
  p[0] = v.x; p[1] = v.y; p[2] = v.z;
}

int orc_evaporate(int A, int Z, double Ex, const double P[3], uint64_t seed, uint64_t event_id,
                  const orc_options* opt_in, orc_result* res, orc_secondary* sec, int sec_cap) {
  if (A < 1 || Z < 0 || Z > A || !(Ex >= 0.0) || !res) return -1;
  orc_nucleus nu;
  std::memset(&nu, 0, sizeof(nu));
  orc_options opt;
  std::memset(&opt, 0, sizeof(opt));
  opt.fixed_b = -1.0;
  if (opt_in) opt.photon_evaporation = opt_in->photon_evaporation;
  if (opt_in) opt.heavy_fragments = opt_in->heavy_fragments;
  std::vector<orc_secondary> out;
  std::memset(res, 0, sizeof(*res));
  Event ev(nu, opt, seed, event_id, *res, out, 0);
  ev.evaporate(A, Z, Ex, {P[0], P[1], P[2]});
  res->n_draw = ev.rng.drawn;
  for (int k = 0; k < (int)out.size() && k < sec_cap; ++k) sec[k] = out[k];
  return (int)out.size();
}

int64_t orc_run(const int* targets_AZ, int n_targets, const orc_options* opt_in, size_t n,
                const uint8_t* tidx, const double* T0, uint64_t seed, uint64_t first_id,
                orc_result* res, orc_secondary* sec, size_t sec_cap, int n_threads) {
  if (!targets_AZ || n_targets < 1 || n_targets > 255 || !T0 || !res) return -1;
  orc_options opt;
  std::memset(&opt, 0, sizeof(opt));
  opt.fixed_b = -1.0;
  if (opt_in) opt = *opt_in;
  std::vector<orc_nucleus> nuclei(n_targets);
  for (int t = 0; t < n_targets; ++t) {
    const int A = targets_AZ[2 * t], Z = targets_AZ[2 * t + 1];
    if (A < 4 || A > 250 || Z < 1 || Z >= A) return -1;
    setup_nucleus(A, Z, opt, nuclei[t]);
  }
  for (size_t i = 0; i < n; ++i) {
    if (tidx && tidx[i] >= n_targets) return -1;
    if (!(T0[i] >= 20.0 && T0[i] <= 250.0)) return -1;
  }
  if (n_threads < 1) n_threads = 1;
  if ((size_t)n_threads > n) n_threads = (int)std::max<size_t>(n, 1);
  std::vector<std::vector<orc_secondary>> outs(n_threads);
  std::vector<std::thread> pool;
  for (int th = 0; th < n_threads; ++th) {
    pool.emplace_back([&, th]() {
      const size_t lo = n * th / n_threads, hi = n * (th + 1) / n_threads;
      for (size_t i = lo; i < hi; ++i) {
        const orc_nucleus& nu = nuclei[tidx ? tidx[i] : 0];
        Event ev(nu, opt, seed, first_id + i, res[i], outs[th], (uint32_t)i);
        ev.run(T0[i]);
      }
    });
  }
  for (auto& t : pool) t.join();
  size_t total = 0;
  for (int th = 0; th < n_threads; ++th) {
    for (const orc_secondary& s : outs[th]) {
      if (sec && total < sec_cap) sec[total] = s;
      ++total;
    }
  }
  return (int64_t)total;
}

}  // extern "C"
