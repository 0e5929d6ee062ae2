// tally.hip — residual-nuclide tally: counts of the final residual (A_f, Z_f)
// per target and incident-energy bin, the reduction behind positron-emitter
// yields (11C, 13N, 15O, ... for range verification, Sec. 4.2 outlook).
#include <hip/hip_runtime.h>

#include "ctx.h"

namespace incdev {

constexpr size_t kTallyLdsMax = 48 * 1024;  // bins kept in LDS below this size

// Bin of T0 among n_ebins equal bins over [20, 250] MeV (FP32, IEEE).
__device__ __forceinline__ int energy_bin(float T0, int n_ebins) {
  const int b = (int)((T0 - 20.0f) * (float)n_ebins / 230.0f);
  return b < 0 ? 0 : (b >= n_ebins ? n_ebins - 1 : b);
}

// Grid-stride over events; a block counts into LDS (32-bit) when the table
// fits there and adds its non-zero bins to the global table at the end,
// otherwise every event adds to the global table directly.  Integer work
// only: the result does not depend on the launch shape.
__global__ void __launch_bounds__(256) k_tally(const inc_residual* res, const float* T0, const uint8_t* tidx,
                                               size_t n, int n_targets, int n_ebins, int amax, int zmax,
                                               unsigned long long* table, int use_lds) {
  extern __shared__ unsigned int bins[];
  const int nb = n_targets * n_ebins * (zmax + 1) * (amax + 1);
  if (use_lds) {
    for (int i = threadIdx.x; i < nb; i += blockDim.x) bins[i] = 0u;
    __syncthreads();
  }
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const inc_residual r = res[i];
    if ((r.flags & 0x8000u) || r.A_f == 0) continue;  // out-of-range input, empty residual
    const int t = tidx ? (int)tidx[i] : 0;
    if (t >= n_targets || r.A_f > amax || r.Z_f > zmax) continue;
    const int k = ((t * n_ebins + energy_bin(T0[i], n_ebins)) * (zmax + 1) + r.Z_f) * (amax + 1) + r.A_f;
    if (use_lds)
      atomicAdd(&bins[k], 1u);
    else
      atomicAdd(&table[k], 1ull);
  }
  if (use_lds) {
    __syncthreads();
    for (int i = threadIdx.x; i < nb; i += blockDim.x)
      if (bins[i]) atomicAdd(&table[i], (unsigned long long)bins[i]);
  }
}

}  // namespace incdev

using namespace incdev;

extern "C" {

int inc_ctx_tally_shape(const inc_ctx* ctx, int* n_targets, int* amax, int* zmax) {
  if (!ctx || !n_targets || !amax || !zmax) return INC_ERR_ARG;
  *n_targets = ctx->n_targets;
  *amax = ctx->amax;
  *zmax = ctx->zmax;
  return INC_OK;
}

int inc_tally_residuals(inc_ctx* ctx, const inc_batch* batch, const inc_residual* res, int n_ebins,
                        unsigned long long* table, void* stream) {
  if (!ctx || !batch || !res || !table || !batch->T0 || batch->n == 0 || batch->n >= (1ull << 32) || n_ebins < 1 ||
      n_ebins > 1024)
    return INC_ERR_ARG;
  const size_t nb = (size_t)ctx->n_targets * n_ebins * (ctx->zmax + 1) * (ctx->amax + 1);
  if (nb >= (1ull << 31)) return INC_ERR_ARG;
  const int use_lds = nb * sizeof(unsigned int) <= kTallyLdsMax;
  const size_t want = (batch->n + 255) / 256;
  const size_t cap = (size_t)ctx->n_cu * 8;
  const unsigned grid = (unsigned)(want < cap ? want : cap);
  hipLaunchKernelGGL(k_tally, dim3(grid), dim3(256), use_lds ? nb * sizeof(unsigned int) : 0, (hipStream_t)stream,
                     res, batch->T0, batch->target_idx, batch->n, ctx->n_targets, n_ebins, ctx->amax, ctx->zmax,
                     table, use_lds);
  return inc_map_hip_error(hipGetLastError());
}

}  // extern "C"
