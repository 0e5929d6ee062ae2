// setup.hip — table kernels run once per context (Sec. 2.2 nucleus, Sec. 2.3
// NN cross-sections, Sec. 2.4 binding energies), shared by both builds of the
// event kernels.
#include "kernels.h"

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

// Evaporation rows (ChanRow) of every (A, Z) of the binding table, with the
// arithmetic the evaporation step would otherwise repeat every step.
__global__ void k_chan_table(const double* B, int amax, int zmax, const EvapTab* et, const MassTab* mt,
                             ChanRow* chan) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int zs = zmax + 1;
  if (idx >= (amax + 1) * zs) return;
  const int A = idx / zs, Z = idx % zs;
  const int fa[6] = {1, 1, 2, 3, 3, 4}, fz[6] = {0, 1, 1, 1, 2, 2};
  const double BAZ = B[idx];
  ChanRow r;
  r.M = (float)((double)Z * kMassP + (double)(A - Z) * kMassN - BAZ);
  // photon channel (option): s0 = 12 N Z / (A E_G^2) fm^2/MeV, the linear
  // photoabsorption ramp up to E_G = 31.2 A^-1/3 + 20.6 A^-1/6 MeV that
  // holds the classical dipole sum 60 N Z / A mb MeV
  if (A >= 2 && Z >= 1 && Z < A) {
    const double EG = 31.2 / cbrt((double)A) + 20.6 / pow((double)A, 1.0 / 6.0);
    r.lg = (float)log(12.0 * (double)(A - Z) * (double)Z / ((double)A * EG * EG) / 3.14159265358979323846);
  } else {
    r.lg = -INFINITY;
  }
  for (int j = 0; j < 6; ++j) {
    const int Ad = A - fa[j], Zd = Z - fz[j];
    if (Z <= A && Ad >= 1 && Zd >= 0 && Zd <= Ad) {
      r.S[j] = (float)(BAZ - B[Ad * zs + Zd] - et->B[j]);
      const float ad13 = mt->a13[Ad];
      r.V[j] = fz[j] ? kE2 * (float)(fz[j] * Zd) / (1.5f * (ad13 + et->a13[j])) : 0.0f;
      const float lnAd = mt->lnA[Ad];
      // ln R_j^2: R_j = 1.5 A_d^1/3 (n, p) or 1.5 (A_d^1/3 + a_j^1/3)
      const float lnR2 = j <= 1 ? 0.8109302f + (2.0f / 3.0f) * lnAd : 2.0f * logf(1.5f * (ad13 + et->a13[j]));
      r.P[j] = et->lngm[j] + lnR2;
    } else {
      r.S[j] = INFINITY;
      r.V[j] = 0.0f;
      r.P[j] = -INFINITY;
    }
  }
  chan[idx] = r;
}

// The heavier fragments' rows (option heavy_fragments, reading R20) for every
// (A, Z) of the binding table, as k_chan_table makes the particles' rows:
// S_j = B(A, Z) - B(A_d, Z_d) - B_j, V_j = e^2 z_j Z_d / (1.5 (A_d^1/3 +
// a_j^1/3)), ln(g_j m_j R_j^2) with R_j = 1.5 (A_d^1/3 + a_j^1/3); and the
// fragments' masses.
__global__ void k_heavy_table(const double* B, int amax, int zmax, const MassTab* mt, HeavyRow* rows,
                              float* hmass) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int zs = zmax + 1;
  if (idx >= (amax + 1) * zs) return;
  const int A = idx / zs, Z = idx % zs;
  constexpr int ha[kHeavy] = INC_HEAVY_A;
  constexpr int hz[kHeavy] = INC_HEAVY_Z;
  constexpr int hg[kHeavy] = INC_HEAVY_G;
  const double BAZ = B[idx];
  HeavyRow r;
  for (int i = 0; i < kHeavy; ++i) {
    const double bj = semf_binding(ha[i], hz[i]);
    const double mj = (double)hz[i] * kMassP + (double)(ha[i] - hz[i]) * kMassN - bj;
    if (idx == 0) hmass[i] = (float)mj;
    const int Ad = A - ha[i], Zd = Z - hz[i];
    if (Z <= A && Ad >= 1 && Zd >= 0 && Zd <= Ad) {
      r.S[i] = (float)(BAZ - B[Ad * zs + Zd] - bj);
      const float R = 1.5f * (mt->a13[Ad] + mt->a13[ha[i]]);
      r.V[i] = kE2 * (float)(hz[i] * Zd) / R;
      r.P[i] = (float)log((double)hg[i] * mj) + 2.0f * logf(R);
    } else {
      r.S[i] = INFINITY;
      r.V[i] = 0.0f;
      r.P[i] = -INFINITY;
    }
  }
  rows[idx] = r;
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
      for (int k = 0; k < 5; ++k) out[t].pad[k] = 0.0f;
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
      const double m = sp ? (double)kMassP : (double)kMassN;
      out[t].EYmax[sp] = (float)sqrt((double)pfmax * (double)pfmax + m * m);
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

// Copy one segment description (a kernel argument) into device memory.
__global__ void k_set_segment(Segment s, Segment* dst) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *dst = s;
}

// ----------------------------------------------------------- start order
// A scheduling choice, not physics: the persistent kernels start the events
// with the largest expected cost first, so that the last events to start are
// short ones and the launch's drain is shorter.  Counting sort: each of
// kOrderBlocks blocks counts the buckets of its slice of the events, two scans
// turn the counts into each (bucket, block) pair's first position, and each
// block scatters its slice from there.  Order within a (bucket, block) pair is
// that of LDS atomics.

// Bucket of event i: 0 for the largest expected cost; a13[t] = A_t^1/3.
__device__ __forceinline__ int order_bin(const float* T0, const uint8_t* tidx, size_t i, const float* a13,
                                         int n_targets, float inv_cmax) {
  const float t = T0[i];
  const int g = tidx ? (int)tidx[i] : 0;
  if (!(t >= 20.0f && t <= 250.0f) || g >= n_targets) return kOrderBins - 1;
  const float c = a13[g] * (t + 50.0f) * inv_cmax;  // (0, 1]
  const int b = (int)((1.0f - c) * (float)kOrderBins);
  return b < 0 ? 0 : (b >= kOrderBins ? kOrderBins - 1 : b);
}
__device__ __forceinline__ void order_slice(size_t n, size_t& lo, size_t& hi) {
  const size_t per = (n + kOrderBlocks - 1) / kOrderBlocks;
  lo = (size_t)blockIdx.x * per;
  hi = lo + per < n ? lo + per : n;
}
// Per block: the targets' A^1/3 in LDS (thread t < n_targets).
__device__ __forceinline__ void order_a13(float* a13, const NucTab* nuc, int n_targets) {
  if ((int)threadIdx.x < n_targets) a13[threadIdx.x] = cbrtf((float)nuc[threadIdx.x].A);
}
// Add one to counter[b] for every active lane, one LDS atomic per distinct
// bucket of the wave (lanes of a wave mostly share a few buckets); returns
// the counter's value before this lane's increment.
__device__ __forceinline__ uint32_t order_bump(uint32_t* counter, int b, bool on) {
  uint32_t mine = 0;
  uint64_t todo = __ballot(on);
  while (todo) {
    const int lead = __ffsll((unsigned long long)todo) - 1;
    const int lb = __shfl(b, lead);
    const uint64_t m = __ballot(on && b == lb);
    uint32_t base = 0;
    if (lane_id() == lead) base = atomicAdd(&counter[lb], (uint32_t)__popcll(m));
    base = (uint32_t)__shfl((int)base, lead);
    if (on && b == lb) mine = base + rank_in(m);
    todo &= ~m;
  }
  return mine;
}
__global__ void __launch_bounds__(256) k_order_count(const float* T0, const uint8_t* tidx, size_t n,
                                                     const NucTab* nuc, int n_targets, float inv_cmax,
                                                     uint32_t* hist) {
  __shared__ uint32_t h[kOrderBins];
  __shared__ float a13[kMaxTargets];
  h[threadIdx.x] = 0u;
  order_a13(a13, nuc, n_targets);
  __syncthreads();
  size_t lo, hi;
  order_slice(n, lo, hi);
  for (size_t i0 = lo; i0 < hi; i0 += blockDim.x) {
    const size_t i = i0 + threadIdx.x;
    const bool on = i < hi;
    (void)order_bump(h, on ? order_bin(T0, tidx, i, a13, n_targets, inv_cmax) : 0, on);
  }
  __syncthreads();
  hist[(size_t)threadIdx.x * kOrderBlocks + blockIdx.x] = h[threadIdx.x];
}
// One block per bucket: the bucket's counts per block become exclusive
// prefixes within the bucket; the bucket's total goes after all rows.
__global__ void __launch_bounds__(kOrderBlocks) k_order_rowscan(uint32_t* hist) {
  __shared__ uint32_t v[kOrderBlocks];
  uint32_t* row = hist + (size_t)blockIdx.x * kOrderBlocks;
  const uint32_t x = row[threadIdx.x];
  v[threadIdx.x] = x;
  __syncthreads();
  for (int d = 1; d < kOrderBlocks; d <<= 1) {  // inclusive scan (Hillis-Steele)
    const uint32_t add = (int)threadIdx.x >= d ? v[threadIdx.x - d] : 0u;
    __syncthreads();
    v[threadIdx.x] += add;
    __syncthreads();
  }
  row[threadIdx.x] = v[threadIdx.x] - x;
  if (threadIdx.x == kOrderBlocks - 1) hist[(size_t)kOrderBins * kOrderBlocks + blockIdx.x] = v[threadIdx.x];
}
// One block: the buckets' totals become the buckets' first positions.
__global__ void __launch_bounds__(kOrderBins) k_order_binscan(uint32_t* hist) {
  __shared__ uint32_t v[kOrderBins];
  uint32_t* tot = hist + (size_t)kOrderBins * kOrderBlocks;
  const uint32_t x = tot[threadIdx.x];
  v[threadIdx.x] = x;
  __syncthreads();
  for (int d = 1; d < kOrderBins; d <<= 1) {
    const uint32_t add = (int)threadIdx.x >= d ? v[threadIdx.x - d] : 0u;
    __syncthreads();
    v[threadIdx.x] += add;
    __syncthreads();
  }
  tot[threadIdx.x] = v[threadIdx.x] - x;
}
__global__ void __launch_bounds__(256) k_order_scatter(const float* T0, const uint8_t* tidx, size_t n,
                                                       const NucTab* nuc, int n_targets, float inv_cmax,
                                                       const uint32_t* hist, uint32_t* perm) {
  __shared__ uint32_t cur[kOrderBins];
  __shared__ float a13[kMaxTargets];
  cur[threadIdx.x] =
      hist[(size_t)kOrderBins * kOrderBlocks + threadIdx.x] + hist[(size_t)threadIdx.x * kOrderBlocks + blockIdx.x];
  order_a13(a13, nuc, n_targets);
  __syncthreads();
  size_t lo, hi;
  order_slice(n, lo, hi);
  for (size_t i0 = lo; i0 < hi; i0 += blockDim.x) {
    const size_t i = i0 + threadIdx.x;
    const bool on = i < hi;
    const uint32_t pos = order_bump(cur, on ? order_bin(T0, tidx, i, a13, n_targets, inv_cmax) : 0, on);
    if (on) perm[pos] = (uint32_t)i;
  }
}

}  // namespace incdev

using namespace incdev;

hipError_t inc_launch_setup(const int* d_AZ, int n_targets, NucTab* d_nuc, XsTab* d_xs, double* d_B, ChanRow* d_chan,
                            int amax, int zmax, EvapTab* d_evap, MassTab* d_mass, const inc_options& o,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_nucleus_setup, dim3(n_targets), dim3(64), 0, s, d_AZ, d_nuc, o.uniform_density, o.zero_fermi,
                     o.zero_binding);
  hipLaunchKernelGGL(k_xs_table, dim3(1), dim3(kXsNodes), 0, s, d_xs, o.const_sigma_mb);
  const int cells = (amax + 1) * (zmax + 1) > kMaxA + 1 ? (amax + 1) * (zmax + 1) : kMaxA + 1;
  hipLaunchKernelGGL(k_bind_table, dim3((cells + 255) / 256), dim3(256), 0, s, d_B, amax, zmax, d_evap, d_mass);
  const int rows = (amax + 1) * (zmax + 1);
  hipLaunchKernelGGL(k_chan_table, dim3((rows + 255) / 256), dim3(256), 0, s, d_B, amax, zmax, d_evap, d_mass,
                     d_chan);
  return hipGetLastError();
}

hipError_t inc_launch_heavy_setup(const double* d_B, int amax, int zmax, const MassTab* d_mass, HeavyRow* d_rows,
                                  float* d_hmass, hipStream_t s) {
  const int rows = (amax + 1) * (zmax + 1);
  hipLaunchKernelGGL(k_heavy_table, dim3((rows + 255) / 256), dim3(256), 0, s, d_B, amax, zmax, d_mass, d_rows,
                     d_hmass);
  return hipGetLastError();
}

hipError_t inc_launch_order(const float* T0, const uint8_t* tidx, size_t n, const NucTab* nuc, int n_targets,
                            float inv_cmax, uint32_t* hist, uint32_t* perm, hipStream_t s) {
  static_assert(kOrderBins == 256, "one thread per bucket");
  hipLaunchKernelGGL(k_order_count, dim3(kOrderBlocks), dim3(256), 0, s, T0, tidx, n, nuc, n_targets, inv_cmax, hist);
  hipLaunchKernelGGL(k_order_rowscan, dim3(kOrderBins), dim3(kOrderBlocks), 0, s, hist);
  hipLaunchKernelGGL(k_order_binscan, dim3(1), dim3(kOrderBins), 0, s, hist);
  hipLaunchKernelGGL(k_order_scatter, dim3(kOrderBlocks), dim3(256), 0, s, T0, tidx, n, nuc, n_targets, inv_cmax, hist,
                     perm);
  return hipGetLastError();
}

hipError_t inc_upload_segment(const Segment& seg, Segment* d_slot, hipStream_t s) {
  hipLaunchKernelGGL(k_set_segment, dim3(1), dim3(64), 0, s, seg, d_slot);
  return hipGetLastError();
}

