// api.hip — the C ABI declared in include/inc.h: context with resident
// tables, argument validation, launch policy and the synchronous host
// convenience call.
#include <string.h>

#include <mutex>
#include <new>

#include "ctx.h"

using namespace incdev;

// Workspace of inc_simulate_dev_noalloc: the hand-over records (plain and
// staged modes), the start order and its counting-sort histogram of one
// launch of at most INC_NOALLOC_MAX_EVENTS events, in static device memory
// (each device holds its own copy from the library's load to the process's
// end).  Host code never passes this name to a kernel: it holds a host-side
// stand-in, not a device address.  Every use goes through the address that
// hipGetSymbolAddress returns for the current device (noalloc_ws).
namespace {
constexpr size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
constexpr size_t kWsMidBytes = align256(mid_bytes(INC_NOALLOC_MAX_EVENTS));
constexpr size_t kWsPermBytes = align256(sizeof(uint32_t) * INC_NOALLOC_MAX_EVENTS);
constexpr size_t kWsHistBytes = align256(sizeof(uint32_t) * kOrderHist);
constexpr size_t kWsBytes = kWsMidBytes + kWsPermBytes + kWsHistBytes;
constexpr int kWsMaxDevices = 64;
}  // namespace
static __device__ __align__(256) unsigned char scratch[kWsBytes];

namespace {

std::mutex ws_mu;
unsigned char* ws_ptr[kWsMaxDevices];  // device address of `scratch`, per device

// Resolve the workspace's address on device `dev` (current) once.
hipError_t noalloc_resolve(int dev) {
  if (dev < 0 || dev >= kWsMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(ws_mu);
  if (ws_ptr[dev]) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!p) return hipErrorInvalidSymbol;
  ws_ptr[dev] = (unsigned char*)p;
  return hipSuccess;
}

// The workspace of device `dev` as launch buffers (resolved by
// inc_ctx_create on that device).
bool noalloc_ws(int dev, Workspace* ws) {
  if (dev < 0 || dev >= kWsMaxDevices) return false;
  unsigned char* p;
  {
    std::lock_guard<std::mutex> g(ws_mu);
    p = ws_ptr[dev];
  }
  if (!p) return false;
  ws->mid = (MidState*)p;
  ws->perm = (uint32_t*)(p + kWsMidBytes);
  ws->hist = (uint32_t*)(p + kWsMidBytes + kWsPermBytes);
  return true;
}

int map_err(hipError_t e) {
  if (e == hipSuccess) return INC_OK;
  if (e == hipErrorOutOfMemory) return INC_ERR_OOM;
  if (e == hipErrorNoDevice || e == hipErrorInvalidDevice) return INC_ERR_NO_DEVICE;
  return INC_ERR_DEVICE;
}

bool valid_target(int A, int Z) { return A >= 4 && A <= 250 && Z >= 1 && Z <= A - 1; }

int current_gfx950(int* dev, int* n_cu) {
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count < 1) return INC_ERR_NO_DEVICE;
  if (hipGetDevice(dev) != hipSuccess) return INC_ERR_NO_DEVICE;
  hipDeviceProp_t p;
  if (hipGetDeviceProperties(&p, *dev) != hipSuccess) return INC_ERR_NO_DEVICE;
  if (strncmp(p.gcnArchName, "gfx950", 6) != 0) return INC_ERR_NO_DEVICE;
  *n_cu = p.multiProcessorCount;
  return INC_OK;
}

void release(inc_ctx* c) {
  if (!c) return;
  if (c->d_nuc) (void)hipFree(c->d_nuc);
  if (c->d_xs) (void)hipFree(c->d_xs);
  if (c->d_mass) (void)hipFree(c->d_mass);
  if (c->d_B) (void)hipFree(c->d_B);
  if (c->d_chan) (void)hipFree(c->d_chan);
  if (c->d_heavy) (void)hipFree(c->d_heavy);
  if (c->d_hmass) (void)hipFree(c->d_hmass);
  if (c->d_mid) (void)hipFree(c->d_mid);
  if (c->d_perm) (void)hipFree(c->d_perm);
  if (c->d_order_hist) (void)hipFree(c->d_order_hist);
  if (c->d_segs) (void)hipFree(c->d_segs);
  if (c->vtx.slots) (void)hipFree(c->vtx.slots);
  if (c->vtx.stacks) (void)hipFree(c->vtx.stacks);
  if (c->vtx.queues) (void)hipFree(c->vtx.queues);
  if (c->vtx.ctl) (void)hipFree(c->vtx.ctl);
  if (c->vtx.h_done) (void)hipHostFree(c->vtx.h_done);
  for (int k = 0; k < 2; ++k)
    if (c->vtx.ev[k]) (void)hipEventDestroy(c->vtx.ev[k]);
  if (c->vtx.capture) (void)hipStreamDestroy(c->vtx.capture);
  delete c;
}

// The vertex pipeline's buffers for a window of the context's vertex_window
// slots (allocated once).
hipError_t ensure_vertex(inc_ctx* ctx) {
  VertexBuf& v = ctx->vtx;
  if (v.slots) return hipSuccess;
  const size_t w = ctx->opt.vertex_window ? (size_t)ctx->opt.vertex_window : (size_t)1 << 18;
  const size_t slot = ctx->opt.fast_math ? fast::vertex_slot_bytes() : precise::vertex_slot_bytes();
  hipError_t e = hipMalloc(&v.slots, slot * w);
  const size_t stack = ctx->opt.fast_math ? fast::vertex_stack_bytes() : precise::vertex_stack_bytes();
  if (e == hipSuccess) e = hipMalloc(&v.stacks, stack * w);
  const size_t qw = ctx->opt.fast_math ? fast::vertex_queue_words(w) : precise::vertex_queue_words(w);
  if (e == hipSuccess) e = hipMalloc(&v.queues, sizeof(uint32_t) * qw);
  if (e == hipSuccess) e = hipMalloc(&v.ctl, sizeof(uint32_t) * kVertexCtlWords);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&v.capture, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipHostMalloc(&v.h_done, sizeof(uint32_t) * 2, hipHostMallocDefault);
  for (int k = 0; k < 2 && e == hipSuccess; ++k) e = hipEventCreateWithFlags(&v.ev[k], hipEventDisableTiming);
  if (e != hipSuccess) {
    if (v.slots) (void)hipFree(v.slots);
    if (v.stacks) (void)hipFree(v.stacks);
    if (v.queues) (void)hipFree(v.queues);
    if (v.ctl) (void)hipFree(v.ctl);
    if (v.h_done) (void)hipHostFree(v.h_done);
    for (int k = 0; k < 2; ++k)
      if (v.ev[k]) (void)hipEventDestroy(v.ev[k]);
    if (v.capture) (void)hipStreamDestroy(v.capture);
    memset(&v, 0, sizeof(v));
    return e;
  }
  v.window = w;
  v.use_graph = ctx->opt.vertex_launch == 0;
  v.cycles_per_group = 8;
  v.max_cycles = 200000;
  return hipSuccess;
}

// The context's hand-over buffer, grown to n events.
hipError_t ensure_mid(inc_ctx* ctx, size_t n) {
  if (ctx->mid_cap >= n) return hipSuccess;
  if (ctx->d_mid) (void)hipFree(ctx->d_mid);
  ctx->d_mid = nullptr;
  ctx->mid_cap = 0;
  hipError_t e = hipMalloc(&ctx->d_mid, mid_bytes(n));
  if (e == hipSuccess) ctx->mid_cap = n;
  return e;
}

// Launch policy and resident tables of a launch of n events.
LaunchDesc launch_desc(const inc_ctx* ctx, size_t n, int mode, int max_blocks) {
  LaunchDesc L;
  memset(&L, 0, sizeof(L));
  L.mode = mode;
  L.block = ctx->block;
  L.persistent_blocks = ctx->n_cu * ctx->waves_per_cu / (ctx->block / 64);
  if (max_blocks > 0 && max_blocks < L.persistent_blocks) L.persistent_blocks = max_blocks;
  if (L.persistent_blocks < 1) L.persistent_blocks = 1;
  L.evap_blocks = ctx->evap_blocks;
  if (max_blocks > 0 && max_blocks < L.evap_blocks) L.evap_blocks = max_blocks;
  L.evap_threshold = ctx->evap_threshold;
  L.tent_threshold = ctx->tent_threshold;
  L.kin_threshold = ctx->kin_threshold;
  L.start_threshold = ctx->start_threshold;
  L.stack_lds = ctx->stack_lds[mode == INC_MODE_PLAIN ? 0 : 1];
  L.chunk = ctx->opt.chunk_events ? ctx->opt.chunk_events : kChunkEvents;
  L.xs_pairs = ctx->opt.table_layout;
  L.photon = ctx->opt.photon_evaporation;
  L.heavy = ctx->opt.heavy_fragments;
  L.heavy_rows = ctx->d_heavy;
  L.heavy_mass = ctx->d_hmass;
  L.nuc = ctx->d_nuc;
  L.n_targets = ctx->n_targets;
  L.xs = ctx->d_xs;
  L.mass = ctx->d_mass;
  L.bind = ctx->d_B;
  L.chan = ctx->d_chan;
  L.amax = ctx->amax;
  L.zmax = ctx->zmax;
  L.evap = ctx->evap;
  L.opt = ctx->opt;
  L.fixed_b_set = ctx->fixed_b_set;
  L.n = n;
  return L;
}

// One segment covering a whole batch with the caller's output buffers.
Segment batch_segment(const inc_output* out, size_t n, uint64_t first_event_id) {
  Segment seg;
  seg.start = 0;
  seg.n = (uint32_t)n;
  seg.first_id = first_event_id;
  seg.res = out->res;
  seg.ev = out->sec_event;
  seg.species = out->sec_species;
  seg.stage = out->sec_stage;
  seg.T = out->sec_T;
  seg.ux = out->sec_ux;
  seg.uy = out->sec_uy;
  seg.uz = out->sec_uz;
  seg.cap = out->sec_capacity;
  seg.counters = out->counters;
  seg.hist = out->history;
  return seg;
}

bool valid_output(const inc_output* out) {
  if (!out || !out->res || !out->counters) return false;
  return !(out->sec_capacity && (!out->sec_event || !out->sec_species || !out->sec_stage || !out->sec_T ||
                                 !out->sec_ux || !out->sec_uy || !out->sec_uz));
}

}  // namespace

int inc_launch_segments(inc_ctx* ctx, size_t n, const uint8_t* tidx, const float* T0, const Segment* d_segs,
                        int n_seg, uint64_t seed, unsigned long long* queue, hipStream_t s, int mode, int max_blocks,
                        const RingDev* ring, MidState* mid, const Workspace* ws) {
  // a launch of the context's own (no hand-over buffer brought by the caller)
  const bool own = !mid;
  if (ws) mid = ws->mid;
  if (!mid && (mode == INC_MODE_PLAIN || mode == INC_MODE_STAGED)) {
    const hipError_t e = ensure_mid(ctx, n);
    if (e != hipSuccess) return map_err(e);
  }
  // the context's own persistent launches start their costliest events first
  const uint32_t* perm = nullptr;
  if (own && (mode == INC_MODE_PERSISTENT || mode == INC_MODE_STAGED || mode == INC_MODE_VERTEX) && n >= kOrderMin &&
      !ctx->opt.input_order) {
    hipError_t e = hipSuccess;
    uint32_t* hist = ws ? ws->hist : ctx->d_order_hist;
    uint32_t* order = ws ? ws->perm : ctx->d_perm;
    if (!ws) {
      if (!ctx->d_order_hist) e = hipMalloc(&ctx->d_order_hist, sizeof(uint32_t) * kOrderHist);
      if (e == hipSuccess && ctx->perm_cap < n) {
        if (ctx->d_perm) (void)hipFree(ctx->d_perm);
        ctx->d_perm = nullptr;
        ctx->perm_cap = 0;
        e = hipMalloc(&ctx->d_perm, sizeof(uint32_t) * n);
        if (e == hipSuccess) ctx->perm_cap = n;
      }
      hist = ctx->d_order_hist;
      order = ctx->d_perm;
    }
    if (e == hipSuccess)
      e = inc_launch_order(T0, tidx, n, ctx->d_nuc, ctx->n_targets, ctx->order_inv_cmax, hist, order, s);
    if (e != hipSuccess) return map_err(e);
    perm = order;
  }
  LaunchDesc L = launch_desc(ctx, n, mode, max_blocks);
  L.perm = perm;
  L.tidx = tidx;
  L.T0 = T0;
  L.segs = d_segs;
  L.n_seg = n_seg;
  L.seed = seed;
  L.queue = queue;
  L.mid = mid ? mid : ctx->d_mid;
  if (ring) L.ring = *ring;
  if (mode == INC_MODE_VERTEX) {
    const hipError_t e = ensure_vertex(ctx);
    if (e != hipSuccess) return map_err(e);
    return map_err(ctx->opt.fast_math ? fast::launch_vertex(L, ctx->vtx, s) : precise::launch_vertex(L, ctx->vtx, s));
  }
  return map_err(ctx->opt.fast_math ? fast::launch_events(L, s) : precise::launch_events(L, s));
}

int inc_launch_batch(inc_ctx* ctx, const inc_batch* b, const inc_output* out, hipStream_t s, int mode, int max_blocks,
                     const Workspace* ws) {
  if (!ctx || !b || !valid_output(out)) return INC_ERR_ARG;
  if (mode != INC_MODE_PLAIN && mode != INC_MODE_PERSISTENT && mode != INC_MODE_STAGED && mode != INC_MODE_VERTEX)
    return INC_ERR_ARG;
  if (mode == INC_MODE_VERTEX && ws) return INC_ERR_ARG;
  if (b->n < 1 || b->n >= (1ull << 32) || !b->T0) return INC_ERR_ARG;
  const Segment seg = batch_segment(out, b->n, b->first_event_id);
  Segment* slot = ctx->d_segs + (ctx->seg_next++ % kSegSlots);
  const int rc = map_err(inc_upload_segment(seg, slot, s));
  if (rc) return rc;
  return inc_launch_segments(ctx, b->n, b->target_idx, b->T0, slot, 1, b->seed, out->counters + 2, s, mode,
                             max_blocks, nullptr, nullptr, ws);
}

int inc_map_hip_error(hipError_t e) { return map_err(e); }

extern "C" {

const char* inc_strerror(int code) {
  switch (code) {
    case INC_OK: return "ok";
    case INC_ERR_ARG: return "invalid argument";
    case INC_ERR_RANGE: return "incident energy outside [20, 250] MeV";
    case INC_ERR_CAPACITY: return "secondary buffer too small";
    case INC_ERR_NO_DEVICE: return "no gfx950 device";
    case INC_ERR_OOM: return "device out of memory";
    case INC_ERR_DEVICE: return "HIP error";
    case INC_ERR_BUSY: return "no free slot or memory now";
    case INC_ERR_TOO_LARGE: return "batch larger than the allocation-free entry point's workspace";
    default: return "unknown error";
  }
}

int inc_contract_version(void) { return 1; }

int inc_ctx_create(const inc_nucleus* targets, int n_targets, const inc_options* opt, inc_ctx** out) {
  if (!out) return INC_ERR_ARG;
  *out = nullptr;
  if (!targets || n_targets < 1 || n_targets > kMaxTargets) return INC_ERR_ARG;
  for (int t = 0; t < n_targets; ++t)
    if (!valid_target(targets[t].A, targets[t].Z)) return INC_ERR_ARG;
  inc_options o;
  memset(&o, 0, sizeof(o));
  if (opt) o = *opt;
  if (o.block_size && (o.block_size < 64 || o.block_size > 256 || o.block_size % 64)) return INC_ERR_ARG;
  if (o.evap_threshold < 0 || o.evap_threshold > 64 || o.tent_threshold < 0 || o.tent_threshold > 64 ||
      o.kin_threshold < 0 || o.kin_threshold > 64 || o.waves_per_cu < 0 || o.waves_per_cu > 32 ||
      o.stack_levels < -1 || o.stack_levels > incdev::kStackLdsMax || o.fast_math < 0 || o.fast_math > 1 ||
      o.start_threshold < 0 || o.start_threshold > 64 || o.input_order < 0 || o.input_order > 1 ||
      o.same_stream < 0 || o.same_stream > 1 || o.photon_evaporation < 0 || o.photon_evaporation > 1 ||
      o.table_layout < 0 || o.table_layout > 1 || o.heavy_fragments < 0 || o.heavy_fragments > 1 ||
      (o.vertex_window && (o.vertex_window < 1024 || o.vertex_window > (1 << 20) ||
                           (o.vertex_window & (o.vertex_window - 1)))) ||
      o.vertex_launch < 0 || o.vertex_launch > 1 ||
      (o.chunk_events && (o.chunk_events < kChunkMin || o.chunk_events > kChunkMax || o.chunk_events % kChunkMin)))
    return INC_ERR_ARG;
  if (!(o.const_sigma_mb >= 0.0f) || o.const_sigma_mb > 1e5f) return INC_ERR_ARG;
  if (o.fixed_b_on && !(o.fixed_b >= 0.0f && o.fixed_b < 20.0f)) return INC_ERR_ARG;
  int dev = 0, n_cu = 0;
  int rc = current_gfx950(&dev, &n_cu);
  if (rc) return rc;
  // the allocation-free entry point's workspace on this device
  if (noalloc_resolve(dev) != hipSuccess) return INC_ERR_DEVICE;

  inc_ctx* c = new (std::nothrow) inc_ctx;
  if (!c) return INC_ERR_OOM;
  memset(c, 0, sizeof(*c));
  c->device = dev;
  c->n_cu = n_cu;
  c->n_targets = n_targets;
  c->opt = o;
  c->fixed_b_set = o.fixed_b_on != 0;
  c->block = o.block_size ? o.block_size : 256;
  // defaults from sweeps on MI355X (16O/40Ca at 200 MeV, staged mode): the
  // tentative-collision and kinematics steps run once 24 lanes wait in them,
  // a flight start once 8 do; 12 resident waves per CU (3 per SIMD)
  c->evap_threshold = o.evap_threshold ? o.evap_threshold : 16;
  c->tent_threshold = o.tent_threshold ? o.tent_threshold : 24;
  c->kin_threshold = o.kin_threshold ? o.kin_threshold : 24;
  c->start_threshold = o.start_threshold ? o.start_threshold : 8;
  c->waves_per_cu = o.waves_per_cu ? o.waves_per_cu : 16;
  int amax = 0, zmax = 0;
  for (int t = 0; t < n_targets; ++t) {
    c->AZ[2 * t] = targets[t].A;
    c->AZ[2 * t + 1] = targets[t].Z;
    amax = targets[t].A + 1 > amax ? targets[t].A + 1 : amax;
    zmax = targets[t].Z + 1 > zmax ? targets[t].Z + 1 : zmax;
  }
  c->amax = amax;
  c->order_inv_cmax = 1.0f / (cbrtf((float)(amax - 1)) * 300.0f);
  c->zmax = zmax;

  int* d_AZ = nullptr;
  EvapTab* d_evap = nullptr;
  hipError_t e = hipSuccess;
  do {
    if ((e = hipMalloc(&c->d_nuc, sizeof(NucTab) * n_targets)) != hipSuccess) break;
    if ((e = hipMalloc(&c->d_xs, sizeof(XsTab))) != hipSuccess) break;
    if ((e = hipMalloc(&c->d_mass, sizeof(MassTab))) != hipSuccess) break;
    if ((e = hipMalloc(&c->d_segs, sizeof(Segment) * kSegSlots)) != hipSuccess) break;
    if ((e = hipMalloc(&c->d_B, sizeof(double) * (amax + 1) * (zmax + 1))) != hipSuccess) break;
    if ((e = hipMalloc(&c->d_chan, sizeof(ChanRow) * (amax + 1) * (zmax + 1))) != hipSuccess) break;
    if ((e = hipMalloc(&d_AZ, sizeof(int) * 2 * n_targets)) != hipSuccess) break;
    if ((e = hipMalloc(&d_evap, sizeof(EvapTab))) != hipSuccess) break;
    if ((e = hipMemcpy(d_AZ, c->AZ, sizeof(int) * 2 * n_targets, hipMemcpyHostToDevice)) != hipSuccess) break;
    if ((e = inc_launch_setup(d_AZ, n_targets, c->d_nuc, c->d_xs, c->d_B, c->d_chan, amax, zmax, d_evap, c->d_mass, o,
                              nullptr)) !=
        hipSuccess)
      break;
    if (o.heavy_fragments) {
      if ((e = hipMalloc(&c->d_heavy, sizeof(HeavyRow) * (amax + 1) * (zmax + 1))) != hipSuccess) break;
      if ((e = hipMalloc(&c->d_hmass, sizeof(float) * kHeavy)) != hipSuccess) break;
      if ((e = inc_launch_heavy_setup(c->d_B, amax, zmax, c->d_mass, c->d_heavy, c->d_hmass, nullptr)) != hipSuccess)
        break;
    }
    if ((e = hipDeviceSynchronize()) != hipSuccess) break;
    e = hipMemcpy(&c->evap, d_evap, sizeof(EvapTab), hipMemcpyDeviceToHost);
    for (int m = 0; m < 2; ++m) {
      const int mode = m == 0 ? INC_MODE_PLAIN : INC_MODE_PERSISTENT;
      const int layout = o.table_layout ? kXsPairs : kXsColumns;
      int lv = o.fast_math ? fast::stack_levels(mode, n_targets, c->block, c->waves_per_cu, layout)
                           : precise::stack_levels(mode, n_targets, c->block, c->waves_per_cu, layout);
      if (o.stack_levels < 0) lv = 0;
      else if (o.stack_levels > 0 && o.stack_levels < lv) lv = o.stack_levels;
      c->stack_lds[m] = lv;
    }
    c->evap_blocks = n_cu * (o.fast_math ? fast::evap_blocks_per_cu(c->block) : precise::evap_blocks_per_cu(c->block));
  } while (false);
  if (d_AZ) (void)hipFree(d_AZ);
  if (d_evap) (void)hipFree(d_evap);
  if (e != hipSuccess) {
    release(c);
    return map_err(e);
  }
  *out = c;
  return INC_OK;
}

int inc_ctx_destroy(inc_ctx* ctx) {
  if (!ctx) return INC_ERR_ARG;
  release(ctx);
  return INC_OK;
}

int inc_ctx_tables(const inc_ctx* ctx, float* host_out) {
  if (!ctx || !host_out) return INC_ERR_ARG;
  NucTab tabs[kMaxTargets];
  hipError_t e = hipMemcpy(tabs, ctx->d_nuc, sizeof(NucTab) * ctx->n_targets, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return map_err(e);
  for (int t = 0; t < ctx->n_targets; ++t) {
    float* o = host_out + 108 * t;
    for (int i = 0; i < kShells; ++i) {
      o[7 * i + 0] = sqrtf(tabs[t].r2[i + 1]);
      o[7 * i + 1] = tabs[t].rho[0][i];
      o[7 * i + 2] = tabs[t].rho[1][i];
      o[7 * i + 3] = tabs[t].pF[0][i];
      o[7 * i + 4] = tabs[t].pF[1][i];
      o[7 * i + 5] = tabs[t].EF[0][i];
      o[7 * i + 6] = tabs[t].EF[1][i];
    }
    o[105] = tabs[t].EB;
    o[106] = tabs[t].EC;
    o[107] = tabs[t].R;
  }
  return INC_OK;
}

int inc_ctx_xs_table(const inc_ctx* ctx, float* host_out, int* n_nodes, float* p_lo, float* p_hi) {
  if (!ctx || !n_nodes || !p_lo || !p_hi) return INC_ERR_ARG;
  static_assert(sizeof(XsTab) == sizeof(float) * 6 * kXsNodes, "six columns of kXsNodes floats");
  *n_nodes = kXsNodes;
  *p_lo = kPlo;
  *p_hi = kPhi;
  if (!host_out) return INC_OK;
  return map_err(hipMemcpy(host_out, ctx->d_xs, sizeof(XsTab), hipMemcpyDeviceToHost));
}

int inc_simulate_dev(inc_ctx* ctx, const inc_batch* b, const inc_output* out, void* stream, int mode) {
  return inc_launch_batch(ctx, b, out, (hipStream_t)stream, mode, 0, nullptr);
}

int inc_simulate_dev_noalloc(inc_ctx* ctx, const inc_batch* b, const inc_output* out, void* stream, int mode) {
  if (!ctx || !b) return INC_ERR_ARG;
  if (b->n > INC_NOALLOC_MAX_EVENTS) return INC_ERR_TOO_LARGE;
  Workspace ws;
  if (!noalloc_ws(ctx->device, &ws)) return INC_ERR_DEVICE;
  return inc_launch_batch(ctx, b, out, (hipStream_t)stream, mode, 0, &ws);
}

int inc_evaporate_dev(inc_ctx* ctx, const inc_excited* in, const inc_output* out, void* stream) {
  if (!ctx || !in || !valid_output(out)) return INC_ERR_ARG;
  if (in->n < 1 || in->n >= (1ull << 32) || !in->A || !in->Z || !in->Ex) return INC_ERR_ARG;
  const hipStream_t s = (hipStream_t)stream;
  hipError_t e = ensure_mid(ctx, in->n);
  if (e != hipSuccess) return map_err(e);
  Segment* slot = ctx->d_segs + (ctx->seg_next++ % kSegSlots);
  e = inc_upload_segment(batch_segment(out, in->n, in->first_event_id), slot, s);
  if (e != hipSuccess) return map_err(e);
  LaunchDesc L = launch_desc(ctx, in->n, INC_MODE_STAGED, 0);
  L.segs = slot;
  L.n_seg = 1;
  L.seed = in->seed;
  L.queue = out->counters + 2;
  L.mid = ctx->d_mid;
  const ExcitedDesc x = {in->A, in->Z, in->Ex, in->P};
  return map_err(ctx->opt.fast_math ? fast::launch_evaporation(L, x, s) : precise::launch_evaporation(L, x, s));
}

int inc_simulate(int target_A, int target_Z, const float* energies, size_t n, uint64_t seed, inc_residual* res,
                 uint32_t* sec_event, uint8_t* sec_species, uint8_t* sec_stage, float* sec_T, float* sec_ux,
                 float* sec_uy, float* sec_uz, size_t cap, size_t* n_sec) {
  if (!energies || !res || !n_sec || n < 1 || n >= (1ull << 32)) return INC_ERR_ARG;
  if (!valid_target(target_A, target_Z)) return INC_ERR_ARG;
  if (cap && (!sec_event || !sec_species || !sec_stage || !sec_T || !sec_ux || !sec_uy || !sec_uz))
    return INC_ERR_ARG;
  for (size_t i = 0; i < n; ++i)
    if (!(energies[i] >= 20.0f && energies[i] <= 250.0f)) return INC_ERR_RANGE;
  inc_nucleus t = {target_A, target_Z};
  inc_ctx* ctx = nullptr;
  int rc = inc_ctx_create(&t, 1, nullptr, &ctx);
  if (rc) return rc;
  const size_t dcap = cap ? cap : 1;
  float* d_T0 = nullptr;
  inc_residual* d_res = nullptr;
  unsigned long long* d_cnt = nullptr;
  char* d_sec = nullptr;
  hipError_t e = hipSuccess;
  unsigned long long cnt[4] = {0, 0, 0, 0};
  const size_t sec_bytes = dcap * (4 + 1 + 1 + 4 * 4);
  do {
    if ((e = hipMalloc(&d_T0, sizeof(float) * n)) != hipSuccess) break;
    if ((e = hipMalloc(&d_res, sizeof(inc_residual) * n)) != hipSuccess) break;
    if ((e = hipMalloc(&d_cnt, sizeof(unsigned long long) * 4)) != hipSuccess) break;
    if ((e = hipMalloc(&d_sec, sec_bytes)) != hipSuccess) break;
    if ((e = hipMemcpy(d_T0, energies, sizeof(float) * n, hipMemcpyHostToDevice)) != hipSuccess) break;
    inc_output o;
    o.res = d_res;
    o.sec_T = (float*)d_sec;
    o.sec_ux = o.sec_T + dcap;
    o.sec_uy = o.sec_ux + dcap;
    o.sec_uz = o.sec_uy + dcap;
    o.sec_event = (uint32_t*)(o.sec_uz + dcap);
    o.sec_species = (uint8_t*)(o.sec_event + dcap);
    o.sec_stage = o.sec_species + dcap;
    o.sec_capacity = cap;
    o.counters = d_cnt;
    o.history = nullptr;
    inc_batch bt = {n, nullptr, d_T0, seed, 0};
    rc = inc_simulate_dev(ctx, &bt, &o, nullptr, INC_MODE_STAGED);
    if (rc) break;
    if ((e = hipDeviceSynchronize()) != hipSuccess) break;
    if ((e = hipMemcpy(cnt, d_cnt, sizeof(cnt), hipMemcpyDeviceToHost)) != hipSuccess) break;
    if ((e = hipMemcpy(res, d_res, sizeof(inc_residual) * n, hipMemcpyDeviceToHost)) != hipSuccess) break;
    const size_t k = cnt[0] < cap ? (size_t)cnt[0] : cap;
    if (k) {
      if ((e = hipMemcpy(sec_T, o.sec_T, 4 * k, hipMemcpyDeviceToHost)) != hipSuccess) break;
      if ((e = hipMemcpy(sec_ux, o.sec_ux, 4 * k, hipMemcpyDeviceToHost)) != hipSuccess) break;
      if ((e = hipMemcpy(sec_uy, o.sec_uy, 4 * k, hipMemcpyDeviceToHost)) != hipSuccess) break;
      if ((e = hipMemcpy(sec_uz, o.sec_uz, 4 * k, hipMemcpyDeviceToHost)) != hipSuccess) break;
      if ((e = hipMemcpy(sec_event, o.sec_event, 4 * k, hipMemcpyDeviceToHost)) != hipSuccess) break;
      if ((e = hipMemcpy(sec_species, o.sec_species, k, hipMemcpyDeviceToHost)) != hipSuccess) break;
      if ((e = hipMemcpy(sec_stage, o.sec_stage, k, hipMemcpyDeviceToHost)) != hipSuccess) break;
    }
  } while (false);
  if (d_T0) (void)hipFree(d_T0);
  if (d_res) (void)hipFree(d_res);
  if (d_cnt) (void)hipFree(d_cnt);
  if (d_sec) (void)hipFree(d_sec);
  inc_ctx_destroy(ctx);
  if (rc) return rc;
  if (e != hipSuccess) return map_err(e);
  *n_sec = (size_t)cnt[0];
  return cnt[0] > cap ? INC_ERR_CAPACITY : INC_OK;
}

}  // extern "C"
