/*
 * fcs.h -- C ABI of the MI355X (gfx950) per-hit calorimeter shower simulator.
 *
 * The method is the parameterized calorimeter simulation ported to GPUs in
 * arXiv 2103.14737: for every particle and calorimeter layer the number of
 * hits is drawn, each hit gets the energy E_layer / nhit (Listing 1 of the
 * CUDA Implementation section), each hit is placed from a random lateral
 * parametrization around the particle position and its cell is looked up,
 * and its energy is added to that cell (Listing 2, HitCellMapping; the
 * sim_a kernel of the same section).  The hit cells are then gathered as
 * {cell_id, E} (the sim_ct kernel) and the workspace is reset (clean).
 *
 * The calls follow the paper's statement of the problem: flatten and load
 * the geometry once and the parametrization tables once (CUDA
 * Implementation section), then run an event loop over particle tuples
 * (type + four-vector, Test Data section) and get back per-event cell
 * energies.  The paper groups the work of many layers, particles and events
 * into one launch (same section, last paragraph); FCS_MODE_BATCHED does that
 * for a whole batch, FCS_MODE_PER_EVENT launches once per event and
 * FCS_MODE_PER_TASK once per (particle, layer), as the paper's first port.
 *
 * Conventions
 *   - Every call returns FCS_OK (0) or a negative FCS_E_* code and never
 *     throws or aborts across the ABI.  fcs_last_error() then describes the
 *     failure (the string lives until the next call on that context).
 *   - Host arrays passed to load calls are copied; the caller keeps
 *     ownership.  Buffers passed to fcs_simulate_events / fcs_backward stay
 *     caller-owned; the library only reads inputs and writes outputs.
 *   - A context is bound to one GPU and is not thread-safe: calls on one
 *     context must be serialized.  Different contexts are independent.
 *   - Units: energies in MeV, lengths in mm, angles in radians, phi in
 *     [-pi, pi).
 */
#ifndef FCS_H
#define FCS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FCS_OK 0
#define FCS_E_INVALID_ARG (-1) /* a malformed argument; message names it   */
#define FCS_E_NOT_LOADED (-2)  /* geometry or parametrization not loaded    */
#define FCS_E_CAPACITY (-3)    /* an output buffer is too small; required
                                  sizes are written to the output struct    */
#define FCS_E_HIP (-4)         /* a HIP runtime call failed                 */
#define FCS_E_NO_DEVICE (-5)   /* no usable GPU                             */
#define FCS_E_NOMEM (-6)       /* device or pinned allocation failed        */

typedef struct fcs_ctx fcs_ctx;

/* ------------------------------------------------------------------------
 * Context
 * ------------------------------------------------------------------------ */

/* Create a context on GPU `device` (HIP ordinal).  *out receives the
 * context; on failure *out is NULL and the code is FCS_E_NO_DEVICE (no GPU
 * or bad ordinal), FCS_E_HIP or FCS_E_NOMEM.  The message of a failed create
 * is available from fcs_last_error(NULL).
 * device = FCS_DEVICE_NONE makes a context without a GPU: every call checks
 * its arguments as usual (loads keep only the shapes) and returns
 * FCS_E_NO_DEVICE where device work would start.  No HIP call is made. */
#define FCS_DEVICE_NONE (-1)
int fcs_create(fcs_ctx **out, int device);

/* Free every device buffer, stream and graph of the context.  NULL is a
 * no-op. */
void fcs_destroy(fcs_ctx *ctx);

/* Description of the last failure on ctx (or of the last failed
 * fcs_create when ctx is NULL).  Never NULL. */
const char *fcs_last_error(const fcs_ctx *ctx);

typedef struct {
    char device_name[64];
    int32_t compute_units;     /* CUs of the device                        */
    int32_t device;            /* HIP ordinal                              */
    int64_t n_cells;           /* loaded geometry, 0 if none               */
    int32_t n_layers;
    int32_t n_regions;
    int64_t n_histograms;      /* loaded parametrization, 0 if none        */
    int64_t device_bytes;      /* device memory held by the context        */
} fcs_info;

int fcs_get_info(const fcs_ctx *ctx, fcs_info *info);

/* Pinned host memory of `bytes` bytes on the context's device (its own
 * allocation, device-writable through its mapping), for the outputs of
 * asynchronous calls that leave their {cell_id, E} lists on the host (see
 * fcs_sim_options.async_launch).  *ptr is NULL on failure (FCS_E_NOMEM,
 * FCS_E_NO_DEVICE for a device-less context).  fcs_host_free waits for the
 * context's copies to the host, then releases it; NULL is a no-op. */
int fcs_host_alloc(fcs_ctx *ctx, int64_t bytes, void **ptr);
int fcs_host_free(fcs_ctx *ctx, void *ptr);

/* ------------------------------------------------------------------------
 * Geometry (CUDA Implementation section: the cell and region data are
 * flattened into arrays and copied to the GPU once).
 *
 * Every layer is cut into n_regions contiguous eta ranges; region k of layer
 * l (index r = l * n_regions + k) is a uniform grid of neta x nphi cells
 * with eta in [eta_lo, eta_hi) and phi in [phi_lo, phi_lo + nphi / inv_dphi).
 * Its cells have dense indices offset + ie * nphi + ip.  A point is in
 * acceptance when eta_lo[first region] <= eta < eta_hi[last region].
 * ------------------------------------------------------------------------ */
typedef struct {
    int64_t n_cells;               /* total cells, = sum of neta * nphi      */
    int32_t n_layers;              /* 1..64                                  */
    int32_t n_regions;             /* regions per layer, 1..8                */
    const int64_t *cell_id;        /* [n_cells] opaque id per dense index    */
    const float *reg_eta_lo;       /* [n_layers * n_regions]                 */
    const float *reg_eta_hi;       /* [n_layers * n_regions]                 */
    const float *reg_inv_deta;     /* 1 / (eta width of a cell)              */
    const float *reg_inv_dphi;     /* 1 / (phi width of a cell)              */
    const float *reg_phi_lo;       /* lower phi edge, normally -pi           */
    const int32_t *reg_neta;       /* cells along eta                        */
    const int32_t *reg_nphi;       /* cells along phi                        */
    const int32_t *reg_offset;     /* dense index of the region's first cell */
    const float *layer_inv_r;      /* [n_layers] 1 / radius (1/mm) of the
                                      layer, converts a lateral offset (mm)
                                      into (deta, dphi)                     */
} fcs_geometry;

/* Copy the geometry to the device (replacing any previous one).  Validated:
 * regions of a layer tile [eta_lo[0], eta_hi[last]) without gaps, offsets
 * are the running sum of neta * nphi, sizes and widths are positive and
 * finite.  FCS_E_INVALID_ARG names the offending field. */
int fcs_load_geometry(fcs_ctx *ctx, const fcs_geometry *geom);

/* ------------------------------------------------------------------------
 * Parametrization (CUDA Implementation section: the tables are flattened
 * and each needed table is loaded to the GPU once).
 *
 * A histogram set is selected per particle from its type, energy and |eta|
 * (Introduction): type t = 0 e+-, 1 photon, 2 pi+- (|pdg| 11, 22, 211),
 * ie = number of e_edges[1..n_ebins-1] <= E, ih = number of
 * eta_edges[1..n_etabins-1] <= |eta|, set = (t * n_ebins + ie) * n_etabins +
 * ih.  Histogram h = set * n_layers + layer has 256 bins b = ir * 8 + ia:
 * 32 radial bins of width r_max_mm / 32 and 8 angular bins of width pi/4.
 * The library stores each histogram as a cumulative FP32 table built from
 * the weights (FP64 running sum over the FP64 total, last entry exactly 1).
 * ------------------------------------------------------------------------ */
typedef struct {
    int32_t n_types;               /* 3                                     */
    int32_t n_ebins;               /* energy bins (16)                      */
    int32_t n_etabins;             /* |eta| bins (10)                       */
    int32_t n_layers;              /* must equal the geometry's             */
    int32_t n_rbins;               /* must be 32                            */
    int32_t n_abins;               /* must be 8                             */
    float r_max_mm;                /* radial extent of the histograms       */
    const float *e_edges;          /* [n_ebins + 1] MeV, increasing         */
    const float *eta_edges;        /* [n_etabins + 1], increasing           */
    const float *dirichlet_alpha;  /* [n_types * n_layers] > 0: per-layer
                                      energy split of a particle of type t */
    const float *weights;          /* [n_sets * n_layers * 256] >= 0, every
                                      histogram with a positive total        */
} fcs_param;

int fcs_load_parametrization(fcs_ctx *ctx, const fcs_param *param);

/* The same load without waiting for the device (the paper's tables were
 * loaded synchronously between calls; here a table change overlaps the
 * batches already running).  The arguments are checked and copied into the
 * library's pinned staging before the call returns, so the caller's arrays
 * may be reused at once.  Upload and table build run on the context's
 * second stream into a second table set, after every call already enqueued
 * on the context; the next fcs_simulate_events / fcs_query_sizes /
 * fcs_backward call makes its stream wait for them (the host does not wait)
 * and uses the new tables, while calls enqueued before keep the old ones
 * (the upload waits only for the calls that may still read the set it
 * overwrites: those enqueued before that set was last switched out).
 * A second asynchronous load first takes the previous one into use; an
 * fcs_load_parametrization supersedes a load not yet taken into use.  The
 * call waits on the host only when the previous asynchronous load's copies
 * are still running or the second set has to grow.  Errors as
 * fcs_load_parametrization. */
int fcs_load_parametrization_async(fcs_ctx *ctx, const fcs_param *param);

/* ------------------------------------------------------------------------
 * Simulation
 * ------------------------------------------------------------------------ */
typedef struct {
    int32_t pdg;    /* 11, 22, 211 (either sign)                             */
    float e_mev;    /* particle energy, finite and > 0                        */
    float eta;      /* finite; |eta| >= 3.2 is simulated, hits fall outside  */
    float phi;      /* finite, in [-pi, pi]                                   */
} fcs_particle;    /* 16 bytes */

#define FCS_MODE_BATCHED 0   /* the whole batch in one persistent launch   */
#define FCS_MODE_PER_EVENT 1 /* one launch sequence + sync per event       */
/* FCS_MODE_PER_TASK: per event, the setup, then the event's hit counts
 * copied to the host and one launch per (particle, layer) task with hits
 * (one thread per hit; each workgroup counts its hits per cell in LDS and
 * adds count x Ehit with one device atomic per cell), then the compaction:
 * the launch structure of the paper's first GPU port (CUDA Implementation
 * section), kept as a baseline; results as in the other modes. */
#define FCS_MODE_PER_TASK 2

#define FCS_OUT_DENSE 1u     /* out->cells                                  */
#define FCS_OUT_COMPACT 2u   /* out->cell_ids / cell_e / event_cell_offsets */
#define FCS_OUT_HITS 4u      /* out->hit_* / task_hit_offsets               */
#define FCS_OUT_COUNTS 8u    /* out->counts                                 */
#define FCS_OUT_ELAYER 16u   /* out->elayer                                 */

typedef struct {
    uint64_t seed;              /* Philox key (low word, high word)          */
    uint64_t event_index_base;  /* global index of event 0 of this batch:
                                   results of an event depend only on
                                   (seed, global index, its particles)      */
    int32_t mode;               /* FCS_MODE_*                                */
    uint32_t outputs;           /* FCS_OUT_* bit set                         */
    float hit_energy_scale_mev; /* expected hits of a layer = E_layer / this */
    int32_t nhit_cap;           /* hits per (particle, layer) are capped     */
    double min_layer_energy_mev;/* layers with less energy get no hits; at
                                   least FLT_MIN x nhit_cap (x 2^26 with
                                   hit_energy_fluct), so that no hit energy
                                   is a subnormal FP32 number               */
    int32_t chunk_hits;         /* tuning, 0 = default: hits per work item of
                                   a large (particle, layer) task, <= 32768 */
    int32_t big_task_hits;      /* tuning, 0 = default: tasks with at least
                                   this many hits are chunked and get a
                                   private cell accumulator                 */
    int32_t tile_hits;          /* tuning, 0 = default: hits per work item of
                                   packed small tasks (>= big_task_hits)    */
    int32_t wg_per_cu;          /* tuning, 0 = default: persistent
                                   workgroups per compute unit              */
    int32_t use_graph;          /* batched mode: capture the launch sequence
                                   in a hipGraph per batch shape and replay */
    int32_t inputs_on_device;   /* particles / event_offsets / override are
                                   device pointers (else host)              */
    int32_t outputs_on_device;  /* every output pointer is a device pointer
                                   (else host; copied back before return)   */
    int32_t profile;            /* 1: time the hit step (window pass and
                                   hit kernel) with HIP events on the stream
                                   it runs on (out->kernel_ms), and in
                                   synchronous calls the setup before it and
                                   the compaction after it (out->setup_ms,
                                   out->compact_ms); the hit step is then
                                   launched outside the captured graph      */
    const float *elayer_override; /* [N * n_layers] or NULL: energies used for
                                   Ehit; hit counts still come from the
                                   particle's own layer energies.  Values
                                   must be finite and >= 0, and a (particle,
                                   layer) with hits must get a hit energy
                                   value / n of at least FLT_MIN (x 2^26
                                   with hit_energy_fluct); else
                                   FCS_E_INVALID_ARG (checked on the device
                                   once the hit counts are known)           */
    void *stream;               /* hipStream_t the call orders after; NULL =
                                   the context's stream                     */
    int64_t n_particles;        /* device inputs: number of records in
                                   particles (checked on the device against
                                   event_offsets[n_events]); 0 = read
                                   event_offsets[n_events] back, one
                                   device-to-host round trip per call       */
    int32_t async_launch;       /* 1: enqueue the batch and return without
                                   waiting (batched mode, device inputs,
                                   n_particles given; device outputs, or
                                   FCS_OUT_COMPACT alone into pinned host
                                   buffers from fcs_host_alloc: then the
                                   batch compacts into one of two device
                                   staging sets used in turn, and a second
                                   stream copies the event offsets and the
                                   lists to the host beside the next
                                   batch's hit kernels (see
                                   host_copy_workgroups): size
                                   cell_capacity to the expected compacted
                                   total.  Host lists are complete after
                                   fcs_synchronize; the copy of a batch is
                                   enqueued by the next call into the
                                   context).  opt->stream is made to wait
                                   for the device results.  The
                                   out->n_* fields are not known and are set
                                   to -1; event_cell_offsets[n_events] holds
                                   the compacted total on the device.
                                   Errors, statistics and hit-kernel times
                                   of async calls are collected by
                                   fcs_synchronize.                         */
    int32_t reuse_forward_queue; /* fcs_backward only: 1 = the caller states
                                   that the particles, offsets and layer
                                   energies hold what they held in the
                                   batched fcs_simulate_events call that
                                   last built the context's work queue.  If
                                   that call took these same device
                                   pointers, options and tuning, and no call
                                   has rebuilt the queue since, the adjoint
                                   reuses it (no setup, no scans); otherwise
                                   the flag has no effect.                  */
    int32_t placement_fp64;      /* fcs_simulate_events: 1 = place every hit
                                   and look up its cell in FP64 (the same
                                   uniforms and bin; cos and sin of the
                                   angle from an FP64 series in turns; the
                                   FP32 geometry values promoted), a chain
                                   variant for measuring how many hits the
                                   FP32 contract puts in another cell.
                                   Hit positions are returned rounded to
                                   FP32.  fcs_backward refuses it
                                   (FCS_E_INVALID_ARG).  Default 0.         */
    int32_t hit_energy_fluct;    /* fcs_simulate_events: 1 = every hit gets
                                   the energy Ehit * x with x = -ln u,
                                   u = ((w >> 8) + 1/2) 2^-24 from the
                                   fourth word of the hit's Philox draw (an
                                   exponential factor of mean 1; x in FP64,
                                   one rounding to FP32): a chain variant
                                   with a per-hit energy stage in place of
                                   the constant Ehit.  A task's energy is
                                   then conserved on average only.  Not
                                   with placement_fp64.  fcs_backward
                                   follows it: dL/dE_l = (1/n) sum over
                                   the task's hits of x g(cell), and the
                                   weight gradient takes each hit's own
                                   energy.  Default 0.                      */
    int32_t window_pass;         /* how the (particle, layer) tasks below
                                   big_task_hits are deposited: 0 = by cell
                                   windows when the launch averages at least
                                   64 particles per event, else in packed
                                   tiles; 1 = by cell windows; -1 = in tiles.
                                   The window pass takes an event, a window
                                   of consecutive cells of one layer and a
                                   range of particles per work item, sums
                                   the hits landing in the window in LDS and
                                   adds them with coalesced atomics.  Not
                                   with placement_fp64, hit_energy_fluct or
                                   FCS_MODE_PER_TASK (tiles then).  Results
                                   as in every other form.                  */
    int32_t window_particles;    /* tuning, 0 = default (1024): particles per
                                   work item of the window pass, 64..65536  */
    int32_t host_copy_workgroups; /* async_launch with host outputs: how the
                                   lists reach the host.  n > 0: a copy
                                   kernel of n workgroups on the second
                                   stream stores the offsets and the
                                   entries the batch wrote (at most
                                   cell_capacity) through the buffers'
                                   device mapping; each workgroup moves
                                   about 25 GB/s (two come near the
                                   link's 56 GB/s), and the link's traffic
                                   slows the kernels beside it, so a batch
                                   whose compute outlasts its copy wants
                                   few.  -1: the runtime's hipMemcpyAsync
                                   of cell_capacity entries.  0 = default
                                   (2 workgroups).  At most 4096.           */
} fcs_sim_options;

/* Fill *opt with the defaults: seed 0, batched, compact output, 100 MeV per
 * hit, cap 20000, 1e-6 MeV minimum layer energy, tuned sizes, graphs on,
 * host inputs and outputs. */
void fcs_default_options(fcs_sim_options *opt);

typedef struct {
    /* FCS_OUT_DENSE: f32 [n_events * n_cells] cell energies (row per event).
       The library zero-fills it first. */
    float *cells;
    /* FCS_OUT_COMPACT: the cells with energy, per event in ascending dense
       index, as (cell_id, E); event e owns [event_cell_offsets[e],
       event_cell_offsets[e+1]).  cell_capacity = entries available. */
    int64_t *cell_ids;
    float *cell_e;
    int64_t *event_cell_offsets;   /* [n_events + 1] */
    int64_t cell_capacity;
    /* FCS_OUT_HITS: one entry per hit in (event, particle, layer, hit)
       order; hit_cell is the dense cell index or -1 outside acceptance;
       task_hit_offsets[t] is the first hit of task t = particle * n_layers +
       layer ([N * n_layers + 1]). */
    float *hit_eta;
    float *hit_phi;
    float *hit_e;
    int32_t *hit_cell;
    int64_t *task_hit_offsets;
    int64_t hit_capacity;
    /* FCS_OUT_COUNTS: i32 [N * n_layers] hits per (particle, layer). */
    int32_t *counts;
    /* FCS_OUT_ELAYER: f32 [N * n_layers] layer energies (MeV). */
    float *elayer;
    /* written by the library */
    int64_t n_hits;                 /* hits generated                        */
    int64_t n_hits_out_of_acceptance;
    int64_t n_tasks;                /* (particle, layer) tasks with hits     */
    int64_t n_cells_nonzero;        /* compacted entries over all events     */
    int64_t required_cell_capacity; /* on FCS_E_CAPACITY                     */
    int64_t required_hit_capacity;
    int64_t n_work_items;           /* chunks + tiles of the last launch     */
    double device_ms;               /* GPU time of the call (hipEvents)      */
    double kernel_ms;               /* with opt->profile: summed duration of
                                       the hit step (window pass and hit
                                       kernel; the per-task launches in
                                       FCS_MODE_PER_TASK).  When the window
                                       pass runs without hit lists it runs
                                       on a second stream beside the task
                                       scans, which then open the hit step */
    double setup_ms;                /* with opt->profile, synchronous calls:
                                       summed duration of the setup pass
                                       (and the task scans when they are not
                                       in the hit step) before the hit step
                                       (-1 for asynchronous calls)           */
    double compact_ms;              /* the same for the compaction and reset
                                       after it                              */
} fcs_sim_output;

/* Simulate n_events events.  particles[N] are grouped by event:
 * event e owns particles [event_offsets[e], event_offsets[e+1]) with
 * event_offsets[0] = 0, non-decreasing, event_offsets[n_events] = N.
 * Deterministic: the hit counts, hit positions and cell indices depend only
 * on (seed, event_index_base + e, the particles), never on the mode, the
 * tuning or the launch shape; cell energies are FP32 sums whose rounding
 * may vary with the order of accumulation.
 * The call returns after the results are complete and copied, unless
 * opt->async_launch is set.
 * Errors: FCS_E_NOT_LOADED, FCS_E_INVALID_ARG (unknown pdg, non-finite or
 * non-positive energy, non-finite eta/phi, bad offsets, missing output
 * pointer), FCS_E_CAPACITY (cell or hit capacity too small: the required
 * sizes are in out->required_*; other outputs are complete), FCS_E_HIP. */
int fcs_simulate_events(fcs_ctx *ctx, const fcs_particle *particles,
                        const int64_t *event_offsets, int64_t n_events,
                        const fcs_sim_options *opt, fcs_sim_output *out);

/* fcs_simulate_events for callers that cannot allocate device memory (code
 * under stream capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same results, but the call allocates nothing.  Every
 * device buffer of the call other than its inputs, its outputs and the
 * loaded tables (the parameter block, counters and work-queue tickets, the
 * per-(particle, layer) arrays, the work queue, the per-block cell counts,
 * the compaction lists and, without FCS_OUT_DENSE, the cell accumulator)
 * is carved from a fixed 64 MiB array in device memory that the library
 * holds on each GPU it runs on until the process ends; no captured graph is
 * used.  Requirements: FCS_MODE_BATCHED, inputs_on_device and
 * outputs_on_device (FCS_E_INVALID_ARG otherwise).  A batch whose workspace
 * does not fit the array fails with FCS_E_INVALID_ARG and a message saying
 * so (about 48 bytes per (particle, layer), 30 KB per event, and 765 KB per
 * event of the 191,338-cell geometry without FCS_OUT_DENSE; split the
 * batch).  The call zeroes the parts of the array that must start at zero.
 * All contexts on one GPU share that GPU's array and each call leaves its
 * contents behind: calls that overlap on one GPU (contexts used from
 * several threads, or an asynchronous call still running when another
 * context's call starts) race and give undefined results.  Calls on one
 * context are ordered on its stream and do not race.  The work queue of
 * such a call is not kept for fcs_backward's reuse_forward_queue. */
int fcs_simulate_events_noalloc(fcs_ctx *ctx, const fcs_particle *particles,
                                const int64_t *event_offsets, int64_t n_events,
                                const fcs_sim_options *opt, fcs_sim_output *out);

/* Statistics of the asynchronous calls since the last fcs_synchronize. */
typedef struct {
    int64_t n_calls;
    int64_t n_hits;
    int64_t n_hits_out_of_acceptance;
    int64_t n_cells_nonzero;
    double kernel_ms;           /* summed hit-step time of profiled calls  */
} fcs_async_stats;

/* Wait for every call enqueued on the context, then report the first error
 * the asynchronous calls met (the codes of fcs_simulate_events; on
 * FCS_E_CAPACITY the outputs of the call that overflowed are incomplete)
 * and, when stats is not NULL, their summed statistics.  Clears both.
 * Synchronous calls need no fcs_synchronize. */
int fcs_synchronize(fcs_ctx *ctx, fcs_async_stats *stats);

typedef struct {
    int64_t n_hits;          /* hits the batch will generate               */
    int64_t n_tasks;         /* (particle, layer) tasks with hits          */
    int64_t max_cells;       /* upper bound of compacted entries           */
} fcs_sizes;

/* Run only the per-(particle, layer) setup of fcs_simulate_events and report
 * the sizes its outputs need. */
int fcs_query_sizes(fcs_ctx *ctx, const fcs_particle *particles,
                    const int64_t *event_offsets, int64_t n_events,
                    const fcs_sim_options *opt, fcs_sizes *sizes);

/* ------------------------------------------------------------------------
 * Adjoint (differentiable form).  Given g = dL/dE_cell as a device f32
 * array [n_events * n_cells] for the batch simulated with the same
 * particles and options, recompute every hit's bin and cell from its Philox
 * counter (nothing is stored by the forward pass) and write
 *   grad_elayer[t] = dL/dE_layer = (1/n_t) sum over the task's in-acceptance
 *                    hits of g[cell]   (hit counts are held fixed),
 *   grad_weights[h*256+b] = A_hb / w_hb - S_h / W_h, the likelihood-ratio
 *                    gradient with samples held at the loaded weights w,
 *                    A_hb = sum over hits of histogram h in bin b of
 *                    g[cell] * Ehit, S_h = sum_b A_hb, W_h = sum_b w_hb
 *                    (A_hb / w_hb is taken as 0 when w_hb = 0).
 * grad_elayer is f32 [N * n_layers], grad_weights f32 [n_histograms * 256]
 * and 16-byte aligned; both are device pointers (either may be NULL).
 * Inputs follow opt->inputs_on_device.  Synchronous like
 * fcs_simulate_events, unless opt->async_launch (device inputs and
 * opt->n_particles required): then the call returns once its work is
 * enqueued, opt->stream (if set) waits for the gradients, and errors are
 * reported by the next fcs_synchronize (adjoint calls are not counted in its
 * statistics).  The context keeps FP64 accumulators for these sums
 * (8 bytes per task and per histogram bin), zeroed when allocated and
 * cleared again by each call.
 * ------------------------------------------------------------------------ */
int fcs_backward(fcs_ctx *ctx, const fcs_particle *particles,
                 const int64_t *event_offsets, int64_t n_events,
                 const fcs_sim_options *opt, const float *grad_cells,
                 float *grad_elayer, float *grad_weights);

#ifdef __cplusplus
}
#endif

#endif /* FCS_H */
