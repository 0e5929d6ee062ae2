/*
 * inc.h — C ABI of the MI355X (gfx950) intranuclear cascade + evaporation
 * library.
 *
 * The library generates proton–nucleus non-elastic events at 20–250 MeV
 * following Wan Chan Tseung & Beltran, "A graphics processor-based intranuclear
 * cascade and evaporation simulation" (arXiv:1309.7963): a Bertini-type
 * cascade in a 15-shell Fermi-gas nucleus (Sec. 2.2, Eq. (1); Sec. 2.3)
 * followed by evaporation of n, p, d, t, 3He and alpha (Sec. 2.4).  Inputs are
 * incident protons (kinetic energy, target) and a random seed; outputs are the
 * escaping and evaporated particles and the residual nucleus (Sec. 3.2, 3.3).
 *
 * Conventions
 *   Units: MeV, MeV/c, fm.  Incident protons move along +z.  Directions are
 *   unit vectors in the target rest frame; T is the asymptotic kinetic energy.
 *   Species codes: 0 n, 1 p, 2 d, 3 t, 4 3He, 5 alpha (options: 6 photon,
 *   7-26 heavier fragments, see inc_options).  Stage 0 = cascade,
 *   1 = evaporation.
 *   Event identity: event i of a batch uses the Philox4x32-10 stream with
 *   key = seed and counter = (block, id lo, id hi, 0), id = first_event_id + i,
 *   so results depend only on (seed, id, target, T0), never on batching.
 *   All functions return 0 (INC_OK) or a negative error code; no exception
 *   crosses the ABI.  Pointers documented as "device" must be device memory
 *   of the current HIP device; "host" pointers are ordinary host memory.
 */
#ifndef INC_H
#define INC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- errors */
#define INC_OK 0
#define INC_ERR_ARG -1        /* invalid argument (target, sizes, pointers)   */
#define INC_ERR_RANGE -2      /* an incident energy outside [20, 250] MeV     */
#define INC_ERR_CAPACITY -3   /* secondary buffer too small; n_sec holds the
                                 required total, residuals are valid          */
#define INC_ERR_NO_DEVICE -4  /* no usable gfx950 device                      */
#define INC_ERR_OOM -5        /* device allocation failed                     */
#define INC_ERR_DEVICE -6     /* a HIP call or kernel launch failed           */
#define INC_ERR_BUSY -7       /* serving: no free slot or HBM budget now      */
#define INC_ERR_TOO_LARGE -8  /* batch larger than inc_simulate_dev_noalloc's
                                 workspace (INC_NOALLOC_MAX_EVENTS events)   */

/* Text of an error code (static storage).  Library plumbing, no passage of
 * the paper. */
const char* inc_strerror(int code);

/* ------------------------------------------------------------- targets */
/* A target nucleus (Sec. 2.2: the nuclear model is built per (A, Z)). */
typedef struct {
  int A; /* mass number, 4 <= A <= 250 */
  int Z; /* charge, 1 <= Z <= A - 1    */
} inc_nucleus;

/* Options.  Zero-initialised = the method as specified, default launch.
 * The hooks reduce the model of Sec. 2.2-2.3 to special cases with closed
 * forms; fast_math is the compiler switch of Sec. 4.2; the launch policy is
 * the scheduling of Sec. 3 (one event per thread) on this hardware. */
typedef struct {
  /* test hooks (special cases with closed-form answers) */
  int uniform_density;   /* every shell at A / (4/3 pi R^3)                  */
  int zero_fermi;        /* p_F = E_F = 0                                    */
  int zero_binding;      /* E_B = E_C = 0                                    */
  int no_pauli;          /* no Pauli test                                    */
  int no_evaporation;    /* stop after the cascade                           */
  int stop_after_first;  /* end the cascade at the first allowed collision  */
  float const_sigma_mb;  /* > 0: every NN cross-section is this constant     */
  int fixed_b_on;        /* 1: every pass enters at impact parameter fixed_b */
  float fixed_b;         /* fm, 0 <= fixed_b < R                             */
  /* launch policy (0 = library default) */
  int block_size;        /* threads per block: 64..256, multiple of 64       */
  int evap_threshold;    /* persistent kernel: lanes waiting in a state that */
  int tent_threshold;    /* make a wave run that state's step next (1..64): */
  int kin_threshold;     /* evaporation, tentative collision, kinematics     */
  int waves_per_cu;      /* persistent kernel: resident waves per CU (0 = 16)*/
  int stack_levels;      /* entries of each lane's LIFO kept in LDS (deeper  */
                         /* ones in private memory): 0 = as many as fit     */
                         /* beside the tables at the launch's occupancy, up */
                         /* to 4; -1 = none; 1..4 = at most that many.      */
                         /* Results do not depend on it.                    */
  /* diagnostics */
  int same_stream;       /* every event of a launch draws from the random    */
                         /* stream of its request's first event id, so all   */
                         /* lanes follow one history (divergence-free rate)  */
  /* arithmetic (Sec. 4.2) */
  int fast_math;         /* 1: event kernels built with approximate          */
                         /* transcendentals (hardware log2, exp2, sqrt),     */
                         /* reciprocal division and flushed FP32 denormals;  */
                         /* results differ from the default in the last bits */
                         /* of each step, so event histories diverge, and    */
                         /* agree with it in distribution                    */
  /* launch policy, continued */
  int start_threshold;   /* persistent kernel: lanes that must wait to begin */
                         /* a flight (entry or stack pop) before the wave    */
                         /* runs that step (1..64; 0 = default)              */
  int input_order;       /* persistent and staged launches of >= 65536      */
                         /* events on a context's own buffers start the      */
                         /* events with the largest expected cost first      */
                         /* (A^1/3 (T0 + 50 MeV), a counting sort on the     */
                         /* device); 1: start them in input order instead.   */
                         /* Results do not depend on it.                     */
  /* model extension (Sec. 2, 2.4) */
  int photon_evaporation; /* 1: photons compete with the six particle       */
                         /* channels at every evaporation step (species 6,   */
                         /* stage 1, T = photon energy): detailed-balance    */
                         /* width with a photoabsorption cross-section      */
                         /* rising linearly to the giant-dipole energy and  */
                         /* holding the classical dipole sum, open while     */
                         /* E* > 0.1 MeV and N Z > 0.  Sec. 2 has excited    */
                         /* nuclei shed energy by particles, then photons;  */
                         /* Sec. 2.4 leaves photons out, so 0 (the default) */
                         /* is the paper's model                             */
  /* launch policy, continued */
  int table_layout;      /* persistent and staged kernels: the NN table in   */
                         /* LDS as columns (0, default: two 4-byte reads per */
                         /* interpolation) or as node pairs (1: entry k of a */
                         /* column holds values k and k+1, one 8-byte read,  */
                         /* twice the LDS, so fewer LIFO levels may fit).    */
                         /* Results do not depend on it.                     */
  int chunk_events;      /* persistent and staged kernels: events a wave     */
                         /* claims from the work queue at once (16..1024, a  */
                         /* multiple of 16; 0 = 64).  Results do not depend  */
                         /* on it.                                           */
  /* model extension (Sec. 2.4), continued */
  int heavy_fragments;   /* 1: the stable isotopes of Li to Mg (6Li 7Li 9Be */
                         /* 10B 11B 12C 13C 14N 15N 16O 17O 18O 19F 20Ne    */
                         /* 21Ne 22Ne 23Na 24Mg 25Mg 26Mg: species 7-26 in  */
                         /* that order) are evaporated too, with the light   */
                         /* particles' width and spectrum and their ground-  */
                         /* state spins.  Sec. 2.4 keeps He and lighter      */
                         /* ejectiles of a model that reaches Mg, so 0 (the */
                         /* default) is the paper's model                    */
  /* launch policy, continued */
  int vertex_window;     /* INC_MODE_VERTEX: events in flight (a power of    */
                         /* two, 1024..2^20; 0 = 2^18).  Each takes about    */
                         /* 2.4 KB of device memory (state and LIFO).        */
                         /* Results do not depend on it.                     */
  int vertex_launch;     /* INC_MODE_VERTEX: each group of 8 cycles goes as  */
                         /* one replay of a graph captured for the call (0, */
                         /* default) or as separate kernel launches (1).     */
                         /* Results do not depend on it.                     */
} inc_options;

/* One residual nucleus per event, 32 bytes: the excited nucleus the cascade
 * leaves (Sec. 2.3, excitation from energy conservation) after its
 * evaporation (Sec. 2.4), the per-event output of Sec. 3.2. */
typedef struct {
  uint16_t A_f, Z_f;     /* final residual                                   */
  uint16_t n_sec;        /* secondaries of this event                        */
  uint16_t flags;        /* 1 stack guard, 2 segment guard, 4 empty residual */
  float Ex_casc;         /* excitation energy after the cascade (MeV)        */
  float Ex_f;            /* excitation energy left after evaporation (MeV)   */
  float p_f[3];          /* final residual momentum (MeV/c)                  */
  uint16_t n_coll;       /* allowed NN collisions in the cascade             */
  uint16_t n_retry;      /* transparent passes before the event (Sec. 2.1)   */
} inc_residual;

/* Device-side output buffers, owned by the caller: the escaping particles of
 * the cascade (Sec. 3.2) and the evaporated particles (Sec. 3.3) as one SoA
 * list of secondaries, and one residual per event. */
typedef struct {
  inc_residual* res;      /* device, n entries (event order)                 */
  uint32_t* sec_event;    /* device, sec_capacity entries: index in batch    */
  uint8_t* sec_species;   /* device, sec_capacity: 0 n, 1 p, 2 d, 3 t, 4 3He,
                             5 alpha, 6 photon (photon_evaporation), 7-26
                             heavier fragments (heavy_fragments)           */
  uint8_t* sec_stage;     /* device, sec_capacity                            */
  float* sec_T;           /* device, sec_capacity: kinetic energy (MeV)      */
  float* sec_ux;          /* device, sec_capacity: direction cosines         */
  float* sec_uy;
  float* sec_uz;
  size_t sec_capacity;
  unsigned long long* counters; /* device, >= 4 entries, caller-owned:
                            [0] secondaries produced (may exceed capacity:
                                only the first sec_capacity are stored),
                            [1] flagged events, [2] and [3] work-queue
                            heads.  Reset by the call.                      */
  uint32_t* history;      /* device, 3 n entries, or NULL (not written):
                            per event [0] the uniforms drawn from its
                            Philox stream (Sec. 3.1), cascade and
                            evaporation together, [1] its cascade's flight
                            segments (Sec. 2.3: one per shell crossing or
                            tentative collision point), [2] where its
                            tentative collisions happened: h = 3 h +
                            shell + 1 over them in order from h = 0, mod
                            2^32 (shells 0..14 from the centre).  All 0
                            for a flagged out-of-range event.  A
                            diagnostic of the event's path, e.g. for
                            comparing replays of one stream               */
} inc_output;

/* A batch of incident protons, in device memory (Sec. 3.2: the input array
 * of incident protons; here kinetic energy and target per event, incidence
 * along +z with the impact point sampled per event). */
typedef struct {
  size_t n;                 /* events, 1 <= n < 2^32                         */
  const uint8_t* target_idx;/* device, n entries into the context's targets;
                               NULL = every event on target 0               */
  const float* T0;          /* device, n kinetic energies in [20, 250] MeV   */
  uint64_t seed;
  uint64_t first_event_id;
} inc_batch;

/* Resident state on one device: nucleus tables, NN table, binding and
 * evaporation tables (Sec. 2.2-2.4; Sec. 3.1 keeps such tables in constant
 * and texture memory). */
typedef struct inc_ctx inc_ctx;

/* Build a context on the current device: nucleus shell tables (Sec. 2.2),
 * the NN cross-section table (Sec. 2.3) and the binding-energy table used by
 * the evaporation (Sec. 2.4) are computed by setup kernels and stay resident.
 * targets: host array of n_targets (1..16) nuclei.  opt: host, may be NULL.
 * The context is not thread-safe: calls on one context must be serialised. */
int inc_ctx_create(const inc_nucleus* targets, int n_targets, const inc_options* opt, inc_ctx** out);
/* Release a context and everything it owns (synchronises the device first
 * through hipFree).  INC_ERR_ARG for NULL. */
int inc_ctx_destroy(inc_ctx* ctx);

/* Copy the context's shell tables (Sec. 2.2, Eq. (1): the 15-shell Fermi
 * density, per-shell Fermi momenta and energies, E_B, E_C) to host memory: for target t, 15 shells x
 * {r_outer, rho_n, rho_p, pF_n, pF_p, EF_n, EF_p} floats, then E_B, E_C, R
 * (108 floats per target).  host_out must hold 108 * n_targets floats. */
int inc_ctx_tables(const inc_ctx* ctx, float* host_out);

/* Copy the context's NN elastic table (Sec. 2.3: the cross-sections, their
 * majorant and the slope of the angular distribution, tabulated for the
 * flights and collisions) to host memory.  *n_nodes receives the number of
 * nodes N and *p_lo, *p_hi the grid's ends (GeV/c): node k sits at
 * p_lab = p_lo (p_hi / p_lo)^(k / (N - 1)), kernels interpolate linearly in
 * log p_lab and clamp outside [p_lo, p_hi].  host_out (NULL: only the sizes
 * are returned) must hold 6 N floats: sigma (mb) of unlike then like pairs,
 * the suffix maximum of sigma over the nodes (the flight majorant) of unlike
 * then like pairs, the slope b ((GeV/c)^-2) of unlike then like pairs.  With
 * const_sigma_mb set, both sigma columns and their maxima hold that value.
 * Synchronous.  Returns INC_ERR_ARG for a NULL context or out-param. */
int inc_ctx_xs_table(const inc_ctx* ctx, float* host_out, int* n_nodes, float* p_lo, float* p_hi);

/* Launch modes (Sec. 3.1-3.3 organise the work as one cascade, then one
 * de-excitation, per thread) */
#define INC_MODE_PLAIN 0      /* one event per thread; cascade kernel then
                                 evaporation kernel (the paper's Sec. 3 shape) */
#define INC_MODE_PERSISTENT 1 /* one fused persistent kernel: lanes refill
                                 from a global work queue                     */
#define INC_MODE_STAGED 2     /* persistent cascade kernel that hands each
                                 post-cascade nucleus and stream position over
                                 in device memory (32 B per event) and, once
                                 its own cascades are over, evaporates the
                                 events it handed over; a persistent
                                 evaporation kernel takes any rest.  Same
                                 results as INC_MODE_PERSISTENT               */
#define INC_MODE_VERTEX 3     /* event-based pipeline (the restructuring Sec.
                                 4.2 suggests): a window of in-flight events
                                 whose state stays in device memory, one
                                 kernel per vertex type (flight segments,
                                 tentative collisions, collision kinematics,
                                 evaporation, refill) over compacted queues,
                                 in cycles; the host checks for the end every
                                 few cycles, so the call returns only when the
                                 batch is done.  Same results as
                                 INC_MODE_PERSISTENT; not with a workspace
                                 (inc_simulate_dev_noalloc), the ring or the
                                 server                                       */

/* Generate batch->n non-elastic events (Sec. 2.1: cascade, Sec. 2.3, then
 * evaporation, Sec. 2.4; inputs and outputs as in Sec. 3.2 and 3.3)
 * asynchronously on `stream` (a
 * hipStream_t; NULL = the default stream).  All batch and output pointers
 * are device pointers.  Incident energies are validated on the device:
 * out-of-range events are skipped and counted in counters[1] with
 * flags = 0x8000 in their residual record; the host wrapper inc_simulate
 * turns that into INC_ERR_RANGE.  Returns INC_ERR_ARG for bad sizes or
 * pointers, INC_ERR_DEVICE if a launch fails.  Plain and staged launches use
 * a hand-over buffer, and persistent and staged launches of >= 65536 events
 * a start-order buffer, that the context owns and grows: launches of one
 * context must not overlap on the device (one stream, or synchronise
 * between streams). */
int inc_simulate_dev(inc_ctx* ctx, const inc_batch* batch, const inc_output* out, void* stream, int mode);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * launch as inc_simulate_dev, with the same kernels, arguments, results and
 * errors, except that the hand-over records, the start order and its
 * histogram live in a static device workspace of the library instead of
 * buffers the context grows, so the call allocates nothing (no hipMalloc,
 * hipFree or allocating library routine).  The workspace holds one launch of
 * at most INC_NOALLOC_MAX_EVENTS events (about 37 MiB, reserved on every
 * device the library is loaded on until the process ends); larger batches
 * return INC_ERR_TOO_LARGE with nothing launched.  All calls on one device
 * share that device's workspace: calls that overlap on the device race (use
 * one stream, or synchronise between streams), also across contexts.
 * Everything the kernels read from the workspace is written first in the
 * same launch, so a call never sees the previous call's contents.  The
 * caller still owns the batch and output buffers.  INC_ERR_ARG as for
 * inc_simulate_dev; INC_ERR_DEVICE if the workspace could not be found on
 * the context's device. */
#define INC_NOALLOC_MAX_EVENTS 1048576
int inc_simulate_dev_noalloc(inc_ctx* ctx, const inc_batch* batch, const inc_output* out, void* stream,
                             int mode);

/* ------------------------------------------------ evaporation alone
 * The de-excitation stage of Sec. 2.4 (Weisskopf-Ewing evaporation of n, p,
 * d, t, 3He and alpha until no channel is open) applied to given excited
 * nuclei, e.g. residuals of another cascade model or fixed-excitation
 * studies. */
typedef struct {            /* all arrays are device memory                  */
  size_t n;                 /* nuclei, 1 <= n < 2^32                         */
  const uint16_t* A;        /* n mass numbers, 1 <= A <= amax                */
  const uint16_t* Z;        /* n charges, 0 <= Z <= min(A, zmax)             */
  const float* Ex;          /* n excitation energies, MeV, [0, 500]          */
  const float* P;           /* 3n momenta (x, y, z per nucleus, MeV/c) in the
                               lab frame, or NULL: every nucleus at rest     */
  uint64_t seed;
  uint64_t first_event_id;
} inc_excited;

/* Evaporate in->n excited nuclei asynchronously on `stream` (device memory
 * throughout).  amax and zmax are those of inc_ctx_tally_shape (the
 * heaviest target + 1 nucleon).  Nucleus i draws from the random stream of
 * (seed, first_event_id + i) from its first draw, the same stream
 * inc_simulate_dev gives event first_event_id + i.  out->res[i] receives the
 * final nucleus (A_f, Z_f, Ex_f, p_f), Ex_casc = the given excitation, n_sec
 * = fragments emitted, n_coll = n_retry = 0.  Fragments go to the secondary
 * arrays with stage 1 and sec_event = i, in emission order within a nucleus.
 * A nucleus outside those ranges, or with a non-finite momentum, is not
 * evaporated: its residual is all zero with flags 0x8000 and it is counted
 * in counters[1].  Capacity overflow behaves as in inc_simulate_dev.  Of the
 * context's options, fast_math and same_stream apply; no_evaporation (a
 * cascade hook) does not.  Uses
 * the context's hand-over buffer: calls on one context must not overlap
 * on the device with each other or with inc_simulate_dev.
 * Returns INC_ERR_ARG for a NULL context, input or output pointer, n out of
 * range or secondary arrays missing while sec_capacity > 0; INC_ERR_OOM /
 * INC_ERR_DEVICE if a buffer cannot be grown or a launch fails. */
int inc_evaporate_dev(inc_ctx* ctx, const inc_excited* in, const inc_output* out, void* stream);

/* Convenience form: synchronous, host arrays; events of Sec. 2.1-2.4 on one
 * target, inputs and outputs of Sec. 3.2-3.3.
 * energies_MeV: host, n_events floats.  Results are copied to host arrays
 * res (n_events) and the secondary arrays (sec_capacity each); *n_sec
 * receives the number of secondaries produced.  Returns INC_ERR_CAPACITY when
 * *n_sec > sec_capacity (residuals are still valid), INC_ERR_RANGE when an
 * energy is outside [20, 250] MeV (nothing is simulated). */
int inc_simulate(int target_A, int target_Z, const float* energies_MeV, size_t n_events,
                 uint64_t seed, inc_residual* res, uint32_t* sec_event, uint8_t* sec_species,
                 uint8_t* sec_stage, float* sec_T, float* sec_ux, float* sec_uy, float* sec_uz,
                 size_t sec_capacity, size_t* n_sec);

/* ------------------------------------------------------------- serving
 * Continuous batching of event batches arriving from a transport stepper.
 * A request is admitted when its buffers (inputs, residuals, secondaries) fit
 * in the HBM budget not yet promised to admitted requests, and queues.
 * Whenever one of max_slots slots (HIP streams of the server) is free, the
 * queued requests sharing the head's seed are launched together as one
 * persistent-kernel launch in which every request keeps its own event ids and
 * output buffers; launches on different slots overlap on the device.  Tables
 * stay resident in the context; a request's results depend only on (seed,
 * first_event_id + i, target, T0), so they are the same alone and in the mix.
 * Progress is made inside the server calls (submit, poll, wait, fetch,
 * replay).  Not thread-safe. */
typedef struct inc_server inc_server;

typedef struct {            /* one request; all pointers are host memory     */
  size_t n;                 /* events, 1 <= n < 2^32                         */
  const uint8_t* target_idx;/* n target indices or NULL                      */
  const float* T0;          /* n energies in [20, 250] MeV (else flagged)    */
  uint64_t seed;
  uint64_t first_event_id;
  size_t sec_capacity;      /* 0 = n min(A, 6 + (A - 1) / 10) + 4096, A the  */
                            /* context's largest target A + 1               */
} inc_request;

typedef struct {            /* host buffers receiving a request's results   */
  inc_residual* res;        /* n entries, or NULL                            */
  uint32_t* sec_event;      /* sec_capacity entries each, or NULL            */
  uint8_t* sec_species;
  uint8_t* sec_stage;
  float *sec_T, *sec_ux, *sec_uy, *sec_uz;
  size_t sec_capacity;
  unsigned long long* n_sec;/* out: secondaries produced, or NULL            */
  double* latency_s;        /* out: submit -> results on host, or NULL       */
} inc_host_output;

/* Counters and latency statistics over the requests completed since the
 * server was created or its statistics were reset.  A request's latency runs
 * from its arrival (its submission; for inc_server_replay, its scheduled
 * arrival time) to its results being on the host. */
typedef struct {
  unsigned long long submitted, completed, rejected_busy, events, secondaries;
  unsigned long long in_flight;   /* admitted, not yet fetched               */
  size_t pool_free_largest;       /* largest free block of the device pool   */
  unsigned long long launches;    /* kernel launches started                 */
  double latency_p50_s;           /* median latency of completed requests    */
  double latency_p99_s;           /* 99th percentile (linear interpolation
                                     between order statistics, position
                                     0.99 (n - 1) of the sorted latencies)  */
  double events_per_s;            /* events of completed requests / (last
                                     completion - first arrival)            */
} inc_server_stats;

/* The serving loop follows the paper's use case (Sec. 1): a transport code
 * hands nuclear-interaction events to the GPU as its protons undergo them, so
 * batches arrive while others run.
 * hbm_budget: bytes of device memory for requests in flight (>= 1 MiB; the
 * server also pins the same amount of host memory); max_slots 1..16.
 * INC_ERR_ARG for bad sizes, INC_ERR_OOM if the pool cannot be allocated. */
int inc_server_create(inc_ctx* ctx, size_t hbm_budget, int max_slots, inc_server** out);
/* Wait for the server's launches, then free its pool, mirror and streams;
 * results not fetched are lost.  INC_ERR_ARG for NULL. */
int inc_server_destroy(inc_server* server);
/* Admit a request (its arrays are copied) or return INC_ERR_BUSY (retry
 * after fetching finished requests); INC_ERR_ARG if it can never fit the
 * budget.  On success *ticket identifies it.  (Sec. 1: one batch of the
 * transport code's nuclear events; Sec. 3.2 inputs.) */
int inc_server_submit(inc_server* server, const inc_request* req, uint64_t* ticket);
/* 1 = results ready on the host, 0 = still running, < 0 error (INC_ERR_ARG:
 * unknown ticket). */
int inc_server_poll(inc_server* server, uint64_t ticket);
/* Block until a request's results are on the host (returns 1).  Returns
 * INC_ERR_BUSY instead of waiting forever when the request is queued and
 * cannot start by itself: the queue is held (inc_server_hold), or nothing is
 * running and the head of the queue does not fit the pool because finished
 * requests have not been fetched.  INC_ERR_ARG: unknown ticket. */
int inc_server_wait(inc_server* server, uint64_t ticket);
/* Copy a ready request's results (out may be NULL to discard) and release
 * its memory; returns the request's status (INC_ERR_CAPACITY when its
 * secondary buffer overflowed, INC_ERR_BUSY if it is not ready yet).
 * Output: Sec. 3.2-3.3 (residual per event, secondaries). */
int inc_server_fetch(inc_server* server, uint64_t ticket, const inc_host_output* out);
/* Fill *out (host) with the statistics above.  INC_ERR_ARG for NULL. */
int inc_server_stats_get(inc_server* server, inc_server_stats* out);
/* Start a new statistics window: counters, latencies and the rate restart
 * from zero (requests in flight are not affected). */
int inc_server_stats_reset(inc_server* server);
/* hold = 1: keep admitting and queueing requests but start no launch; hold =
 * 0: release the queue (it is launched at once, as slots free up).  For a
 * caller that hands over a burst of batches, e.g. all nuclear events of one
 * transport step (Sec. 1), and wants them batched into as few launches as
 * possible.  A launch carries at most 65535 requests.  INC_ERR_ARG for a
 * NULL server or hold outside {0, 1}. */
int inc_server_hold(inc_server* server, int hold);
/* Native request loop: request k arrives arrival_s[k] seconds (ascending)
 * after the call starts; requests are admitted first come first served as
 * memory frees up, batched into launches as slots free up, polled, fetched
 * and discarded.  latency_s[k] receives arrival -> results on host; *span_s
 * the time from the first arrival to the last completion.  The server's
 * statistics cover these requests too (latency from the scheduled arrival). */
int inc_server_replay(inc_server* server, int n_req, const double* arrival_s, const inc_request* reqs,
                      double* latency_s, double* span_s);

/* ------------------------------------------------------------- ring output
 * Streaming output for large batches: the secondaries flow through a ring of
 * `slots` records (a power of two >= 1024) while the kernel runs; the calling
 * thread drains the ring into the caller's host arrays (in ring order) and
 * hands the space back.  A full ring makes the producing waves wait (up to
 * ~3 s without consumer progress, then the call fails with INC_ERR_DEVICE);
 * no record is lost or duplicated.  The ring lives in coherent host memory
 * (inc_ring_create: each record crosses PCIe as a wave stores it) or in
 * device memory (inc_ring_create_device: complete chunks are copied to a
 * pinned host mirror by asynchronous copies on the ring's own stream). */
/* (Sec. 3.2-3.3: the secondaries of the batch, streamed.) */
typedef struct inc_ring inc_ring;

typedef struct {
  unsigned long long records;    /* secondaries that passed through the ring */
  unsigned long long slots;
  unsigned long long wraps;      /* records / slots                           */
  unsigned long long consumer_idle_polls;
  double seconds;                /* launch to last record drained             */
  unsigned int producer_gave_up; /* 1 if a wave timed out waiting for room    */
} inc_ring_stats;

/* Ring of `slots` records (power of two, 1024..2^30) in pinned coherent host
 * memory (7 x 4 bytes per slot) for batches of `ctx`.  INC_ERR_ARG for bad
 * sizes, INC_ERR_OOM if the host memory cannot be pinned. */
int inc_ring_create(inc_ctx* ctx, size_t slots, inc_ring** out);
/* Ring of `slots` records in device memory (6 x 4 bytes per slot), cut into
 * chunks of `chunk` slots (a power of two, 1024..slots/2), with a pinned host
 * mirror of the same size (7 x 4 bytes per slot) and a copy stream of its
 * own (default priority).  The device marks a chunk complete once all of its
 * records are written (and visible in device memory); the calling thread
 * then queues its copy to the mirror and hands it on when the copy is done.
 * The last, incomplete chunk of a batch is copied once the kernel has ended.
 * Used with inc_ring_simulate / inc_ring_simulate_to like a host ring.
 * INC_ERR_ARG for bad sizes, INC_ERR_OOM if memory cannot be allocated. */
int inc_ring_create_device(inc_ctx* ctx, size_t slots, size_t chunk, inc_ring** out);
/* Free a ring (no call may be running on it).  INC_ERR_ARG for NULL. */
int inc_ring_destroy(inc_ring* ring);
/* Generate batch->n events (device inputs, as inc_simulate_dev) with their
 * residuals written to d_res (device, n entries) and their secondaries
 * streamed through the ring into out (host arrays, out->sec_capacity each;
 * *out->n_sec receives the total).  If out->res is not NULL the residuals
 * are also copied there (n entries; from pinned host memory the copy
 * overlaps the drain).  Blocks until the batch is drained.
 * Returns INC_ERR_CAPACITY if the host arrays were too small (the rest was
 * drained and dropped).  Not thread-safe; one call at a time per ring. */
int inc_ring_simulate(inc_ring* ring, const inc_batch* batch, inc_residual* d_res, const inc_host_output* out,
                      void* stream, int mode, inc_ring_stats* stats);

/* One run of consecutive records handed to a ring consumer (Sec. 3.2, 3.3:
 * the secondaries of the batch).  The arrays point into the ring's pinned
 * host memory and are valid only during the callback; their slots go back
 * to the producer when it returns. */
typedef struct {
  unsigned long long first; /* index of the run's first record in the batch's
                               output sequence (runs arrive in order,
                               without gaps)                                  */
  size_t n;                 /* records in the run                             */
  const uint32_t* event;    /* n indices of the event in the batch            */
  const uint32_t* kind;     /* n words: species in bits 0-7, stage in bits
                               8-15 (higher bits are internal)                */
  const float* T;           /* n kinetic energies (MeV)                       */
  const float* ux;          /* n direction cosines                            */
  const float* uy;
  const float* uz;
} inc_ring_chunk;

typedef void (*inc_ring_consumer)(const inc_ring_chunk* chunk, void* user);

/* As inc_ring_simulate, but every run of records is handed to consumer(chunk,
 * user) on the calling thread as it becomes ready, so the output needs no
 * host array sized by the batch (a consumer may histogram, filter or write
 * the records out).  h_res: host, n residuals, or NULL.  *n_sec receives the
 * number of records produced.  A slow consumer makes the producer wait, as
 * a full ring does.  The kernel may be waiting for the consumer to return,
 * so the consumer must not call into this ring, nor make or cause HIP calls
 * that wait for the device (hipFree, device, stream or event
 * synchronisation): they would stall both sides until the producer's
 * bounded wait fails the call with INC_ERR_DEVICE.  Returns
 * INC_ERR_ARG for a NULL ring, batch, d_res, consumer or n_sec. */
int inc_ring_simulate_to(inc_ring* ring, const inc_batch* batch, inc_residual* d_res, inc_residual* h_res,
                         inc_ring_consumer consumer, void* user, unsigned long long* n_sec, void* stream,
                         int mode, inc_ring_stats* stats);

/* ------------------------------------------------------ nuclide tally
 * Residual-nuclide counts, the reduction behind positron-emitter yields
 * (11C, 13N, 15O, 30P, 38K ... for range verification: the application the
 * paper's Sec. 4.2 looks ahead to). */

/* Shape of the context's tally table: n_targets, and the largest residual
 * mass number and charge a context can produce (amax = max A + 1, zmax =
 * max Z + 1 over its targets).  Host out-params. */
int inc_ctx_tally_shape(const inc_ctx* ctx, int* n_targets, int* amax, int* zmax);

/* Add one count per event of a generated batch to
 *   table[((t * n_ebins + e) * (zmax + 1) + Z_f) * (amax + 1) + A_f]
 * with t the event's target index (batch->target_idx, NULL = 0) and e the bin
 * of its incident energy among n_ebins (1..1024) equal bins over [20, 250] MeV
 * (e = (int)((T0 - 20) * n_ebins / 230) in FP32, clamped to the last bin).
 * Events whose residual is flagged out of range (0x8000) or empty (A_f = 0)
 * are not counted.  batch: as given to inc_simulate_dev (seed and ids are not
 * used); res: device, batch->n residuals; table: device, n_targets * n_ebins *
 * (zmax + 1) * (amax + 1) counters owned by the caller, accumulated (zero it
 * before the first batch).  Asynchronous on `stream`.  Returns INC_ERR_ARG
 * for bad pointers or sizes, INC_ERR_DEVICE if the launch fails. */
int inc_tally_residuals(inc_ctx* ctx, const inc_batch* batch, const inc_residual* res, int n_ebins,
                        unsigned long long* table, void* stream);

/* Library version of the frozen physics readings of Sec. 2 (changes when any
 * reading that affects results changes). */
int inc_contract_version(void);

#ifdef __cplusplus
}
#endif
#endif
