// ctx.h — the context object shared by the C ABI (api.hip) and the serving
// loop (server.hip): resident tables and launch policy.
#pragma once

#include "kernels.h"

struct inc_ctx {
  int device;
  int n_targets;
  int AZ[2 * incdev::kMaxTargets];
  inc_options opt;
  bool fixed_b_set;
  incdev::NucTab* d_nuc;
  incdev::XsTab* d_xs;
  incdev::MassTab* d_mass;
  double* d_B;
  incdev::ChanRow* d_chan;  // evaporation rows of every (A, Z) of d_B
  incdev::HeavyRow* d_heavy;  // option heavy_fragments: the heavier fragments' rows (NULL when off)
  float* d_hmass;             // and their masses
  int amax, zmax;
  incdev::EvapTab evap;
  incdev::MidState* d_mid;
  size_t mid_cap;
  uint32_t* d_perm;        // start order of the context's own launches (grown on demand)
  size_t perm_cap;
  uint32_t* d_order_hist;  // kOrderBins x kOrderBlocks counting-sort scratch
  float order_inv_cmax;    // 1 / (largest A^1/3 of the targets x 300 MeV)
  incdev::Segment* d_segs;  // kSegSlots single-segment descriptors, used in turn
  unsigned seg_next;
  int n_cu;
  int block, evap_threshold, tent_threshold, kin_threshold, start_threshold, waves_per_cu;
  int stack_lds[2];  // LIFO entries per lane in LDS: [plain, persistent]
  int evap_blocks;   // staged mode: evaporation kernel grid (full occupancy)
  incdev::VertexBuf vtx;  // INC_MODE_VERTEX buffers (allocated on first use; slots NULL until then)
};


constexpr int kSegSlots = 64;  // inc_simulate_dev calls that may be in flight per context

// Launch buffers that a caller brings instead of the context's own (grown on
// demand): hand-over records for n events (plain and staged modes), the start
// order (n entries) and its kOrderHist-count histogram.
struct Workspace {
  incdev::MidState* mid;
  uint32_t* perm;
  uint32_t* hist;
};

// Launch n events described by n_seg device segments (sorted by start, each
// with its own ids and outputs) that share the random-stream key `seed`;
// queue: two device work-queue counters.
// ring: streaming output of the secondaries (NULL: the segments' arrays).
// mid: plain/staged hand-over buffer of n records (NULL: the context's own,
// grown on demand; launches that overlap on different streams must each
// bring their own).
// ws: every launch buffer comes from ws and nothing is allocated (mid must be
// NULL; the start order is used as for the context's own launches).
__attribute__((visibility("hidden"))) int inc_launch_segments(inc_ctx* ctx, size_t n, const uint8_t* tidx,
                                                              const float* T0, const incdev::Segment* d_segs,
                                                              int n_seg, uint64_t seed, unsigned long long* queue,
                                                              hipStream_t s,
                                                              int mode, int max_blocks,
                                                              const incdev::RingDev* ring = nullptr,
                                                              incdev::MidState* mid = nullptr,
                                                              const Workspace* ws = nullptr);

// Launch one batch (validated like inc_simulate_dev); max_blocks > 0 caps the
// persistent grid (small batches use fewer blocks); ws as for
// inc_launch_segments.  Internal to the library.
__attribute__((visibility("hidden"))) int inc_launch_batch(inc_ctx* ctx, const inc_batch* b,
                                                           const inc_output* out, hipStream_t s, int mode,
                                                           int max_blocks, const Workspace* ws = nullptr);
__attribute__((visibility("hidden"))) int inc_map_hip_error(hipError_t e);
