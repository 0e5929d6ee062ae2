// kernels.h — host-visible launch interface between the C ABI (api.hip) and
// the kernels (kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/inc.h"
#include "device.h"

namespace incdev {

// State handed from the plain cascade kernel to the plain evaporation kernel
// (32 bytes per event).
struct MidState {
  int16_t A, Z;
  uint16_t flags, ncoll, nretry, nsec;
  float E;
  float P[3];
  uint32_t drawn;   // uniforms consumed by the cascade
};
static_assert(sizeof(MidState) == 32, "MidState layout");

// Events per work-queue chunk of the persistent kernels: the default, and
// the range of the chunk_events option (multiples of kChunkMin).
constexpr int kChunkEvents = 64;
constexpr int kChunkMin = 16;
constexpr int kChunkMax = 1024;

// LDS layouts of the NN table in the event kernels: none (evaporation
// kernels), columns (XsLds) or node pairs (XsPairs).
constexpr int kXsNone = -1, kXsColumns = 0, kXsPairs = 1;
__host__ __device__ constexpr size_t xs_lds_bytes(int layout) {
  return layout == kXsPairs ? sizeof(XsPairs) : layout == kXsColumns ? sizeof(XsLds) : 0;
}

// Hand-over buffer of a plain or staged launch of n events: n MidState
// records, then (staged) the chunks whose evaporation is left to the
// evaporation kernel: [0] chunks listed, [1] chunks claimed by the
// evaporation kernel, [2], [3] unused, then the first event of each listed
// chunk (room for chunks as small as kChunkMin).
constexpr size_t mid_bytes(size_t n) {
  return sizeof(MidState) * n + sizeof(uint32_t) * (4 + (n + kChunkMin - 1) / kChunkMin);
}

struct LaunchDesc {
  int mode;
  int block;
  int persistent_blocks;
  int evap_blocks;       // staged mode: grid of the evaporation kernel
  int evap_threshold, tent_threshold, kin_threshold, start_threshold;
  int stack_lds;         // stack entries per lane held in LDS (stack_levels)
  int chunk;             // events per work-queue claim (0: kChunkEvents)
  int xs_pairs;          // persistent kernels: NN table in LDS as node pairs
  int photon;            // the evaporation has the photon channel (instantiation)
  int heavy;             // the evaporation has the heavier fragments (instantiation)
  const NucTab* nuc;
  int n_targets;
  const XsTab* xs;
  const MassTab* mass;
  const double* bind;
  const ChanRow* chan;
  const HeavyRow* heavy_rows;  // option heavy_fragments (NULL when off)
  const float* heavy_mass;
  int amax, zmax;
  EvapTab evap;
  inc_options opt;
  bool fixed_b_set;
  size_t n;
  const uint8_t* tidx;
  const float* T0;
  const Segment* segs;   // device
  int n_seg;
  uint64_t seed;         // random-stream key shared by all segments
  unsigned long long* queue;  // two work-queue heads: [0] cascade, [1] evaporation
  const uint32_t* perm;  // start order of the events (NULL: input order)
  MidState* mid;
  RingDev ring;          // rec == NULL: records go to the segments' arrays
};

// Excited nuclei of an evaporation-only launch (device arrays, see
// inc_excited).
struct ExcitedDesc {
  const uint16_t* A;
  const uint16_t* Z;
  const float* Ex;
  const float* P;  // 3 per nucleus, or NULL (at rest)
};
constexpr float kMaxExcitation = 500.0f;  // MeV

// The event kernels exist in two builds of one source (kernels.hip): IEEE
// arithmetic and precise transcendentals (precise, the default) and the
// fast-math build (fast, Sec. 4.2).  Each namespace provides:
//   lds_bytes     dynamic LDS of an event kernel launch (xs_layout: kXsNone for
//                 the evaporation kernels, else the NN table's layout);
//   stack_levels  LIFO entries per lane that fit in LDS for the event kernel of
//                 `mode` at this block size when `waves_per_cu` waves are meant
//                 to share a CU, with the NN table in xs_layout (the plain
//                 kernel always uses columns; the kernel's own occupancy limit
//                 applies too); 0 when none fit;
//   evap_blocks_per_cu  resident blocks per CU of the staged evaporation
//                 kernel (its own occupancy: it needs fewer registers);
//   launch_events zero the counters, then launch the event kernel(s) of L.mode.
//   launch_evaporation  evaporation alone of L.n given excited nuclei
//                 (L.mid: the hand-over buffer; L.T0, L.tidx unused).
// Device and host buffers of the vertex pipeline (INC_MODE_VERTEX): a window
// of in-flight event slots (vertex_slot_bytes() each), their LIFOs
// (vertex_stack_bytes() each), the stage queues (vertex_queue_words(window))
// and the control words; two pinned done flags and two events for the host's
// checks; a stream to capture a group of cycles as a graph on.
constexpr int kVertexCtlWords = 40;
struct VertexBuf {
  void* slots;
  void* stacks;
  uint32_t* queues;
  uint32_t* ctl;
  size_t window;
  uint32_t* h_done;
  hipEvent_t ev[2];
  hipStream_t capture;
  int use_graph;
  int cycles_per_group;
  long max_cycles;
};

namespace precise {
size_t vertex_slot_bytes();
size_t vertex_stack_bytes();  // one slot's LIFO
size_t vertex_queue_words(size_t window);
hipError_t launch_vertex(const LaunchDesc& L, const VertexBuf& vb, hipStream_t s);
size_t lds_bytes(int n_targets, int block, int xs_layout, int stack_levels);
int stack_levels(int mode, int n_targets, int block, int waves_per_cu, int xs_layout);
int evap_blocks_per_cu(int block);
hipError_t launch_events(const LaunchDesc& L, hipStream_t s);
hipError_t launch_evaporation(const LaunchDesc& L, const ExcitedDesc& x, hipStream_t s);
}  // namespace precise
namespace fast {
size_t vertex_slot_bytes();
size_t vertex_stack_bytes();  // one slot's LIFO
size_t vertex_queue_words(size_t window);
hipError_t launch_vertex(const LaunchDesc& L, const VertexBuf& vb, hipStream_t s);
size_t lds_bytes(int n_targets, int block, int xs_layout, int stack_levels);
int stack_levels(int mode, int n_targets, int block, int waves_per_cu, int xs_layout);
int evap_blocks_per_cu(int block);
hipError_t launch_events(const LaunchDesc& L, hipStream_t s);
hipError_t launch_evaporation(const LaunchDesc& L, const ExcitedDesc& x, hipStream_t s);
}  // namespace fast

}  // namespace incdev

hipError_t inc_launch_setup(const int* d_AZ, int n_targets, incdev::NucTab* d_nuc, incdev::XsTab* d_xs, double* d_B,
                            incdev::ChanRow* d_chan, int amax, int zmax, incdev::EvapTab* d_evap,
                            incdev::MassTab* d_mass, const inc_options& o, hipStream_t s);
// The heavier fragments' rows (option heavy_fragments) after inc_launch_setup
// has filled the binding and mass tables.
hipError_t inc_launch_heavy_setup(const double* d_B, int amax, int zmax, const incdev::MassTab* d_mass,
                                  incdev::HeavyRow* d_rows, float* d_hmass, hipStream_t s);
hipError_t inc_upload_segment(const incdev::Segment& seg, incdev::Segment* d_slot, hipStream_t s);

// Longest-expected-first start order of a launch's n events: perm (device, n
// entries) receives the event indices, largest expected cost first (cost ~
// A^1/3 (T0 + 50 MeV) in kOrderBins buckets; inv_cmax = 1 / the largest
// cost of the context's targets).  hist: device scratch of kOrderHist counts.
// Invalid inputs go last.
namespace incdev {
constexpr int kOrderBins = 256;
constexpr int kOrderBlocks = 512;
constexpr size_t kOrderHist = (size_t)kOrderBins * (kOrderBlocks + 1);
constexpr size_t kOrderMin = 65536;  // smaller launches start in input order
}  // namespace incdev
hipError_t inc_launch_order(const float* T0, const uint8_t* tidx, size_t n, const incdev::NucTab* nuc, int n_targets,
                            float inv_cmax, uint32_t* hist, uint32_t* perm, hipStream_t s);
